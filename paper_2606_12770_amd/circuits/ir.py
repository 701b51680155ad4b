"""Gate IR: the op list a circuit is handed over in.

One op is a 40-byte little-endian record (numpy dtype ``OP_DTYPE``), the same
bytes the C ABI reads as ``sv_op``:

    kind      u32   one of the kind codes below
    target    u32   target qubit, or the lowest qubit of a register (INC/DEC),
                    or the signal qubit (PROJPHASE), or the first qubit (SWAP)
    width     u32   register width (INC/DEC) or the second qubit (SWAP); else 0
    flags     u32   reserved, 0
    ctrl_mask u64   bit j set  <=>  qubit j is a control
    ctrl_val  u64   required value of each control bit (subset of ctrl_mask)
    param     u64   offset into the float64 parameter pool

Qubit j is bit j of the amplitude index (little-endian).  A gate with controls
acts only on basis states i with ``(i & ctrl_mask) == ctrl_val``; a zero bit of
``ctrl_val`` under a set bit of ``ctrl_mask`` is an open (negative) control.

Kinds and their parameters:

    U         2x2 complex matrix, 8 doubles (u00, u01, u10, u11 as re, im);
              new (a0, a1) = U (a0, a1) on each amplitude pair that differs
              only in the target bit, a0 having the target bit 0
    X         no parameter; exchanges the two amplitudes of each pair
    PHASE     1 double theta; multiplies by exp(i theta) where target bit = 1
    RY        1 double theta; U = [[c, -s], [s, c]], c = cos(theta/2),
              s = sin(theta/2), i.e. exp(-i theta Y / 2)
    INC       no parameter; register value v of qubits [target, target+width)
              becomes (v + 1) mod 2^width
    DEC       as INC with (v - 1) mod 2^width
    SWAP      no parameter; exchanges qubits target and width
    PROJPHASE 1 double theta; the projector-controlled phase of a QSVT step:
              with z = [(i & ctrl_mask) == ctrl_val] and s = bit `target` of i,
              multiplies by exp(i theta (1 - 2 (s xor z))).  It equals the
              three-gate sequence  MCX(ctrl -> target) . diag(e^{i theta},
              e^{-i theta}) on target . MCX(ctrl -> target)  (QSVT circuit
              figure, Sec. II.D.5).  Here ctrl_* is a condition, not a control.
"""
from __future__ import annotations

import numpy as np

OP_DTYPE = np.dtype([
    ("kind", "<u4"), ("target", "<u4"), ("width", "<u4"), ("flags", "<u4"),
    ("ctrl_mask", "<u8"), ("ctrl_val", "<u8"), ("param", "<u8"),
])
assert OP_DTYPE.itemsize == 40

U, X, PHASE, RY, INC, DEC, SWAP, PROJPHASE = range(8)
KIND_NAMES = ["U", "X", "PHASE", "RY", "INC", "DEC", "SWAP", "PROJPHASE"]

_H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)


def _ctrl_bits(controls):
    """controls: None, an iterable of qubits (value 1), or a dict qubit->0/1."""
    mask = 0
    val = 0
    if controls is None:
        return 0, 0
    items = controls.items() if isinstance(controls, dict) else ((q, 1) for q in controls)
    for q, v in items:
        q = int(q)
        if mask >> q & 1:
            raise ValueError(f"control qubit {q} given twice")
        mask |= 1 << q
        if v:
            val |= 1 << q
    return mask, val


class Circuit:
    """An append-only gate list on ``n`` qubits plus its parameter pool."""

    def __init__(self, n: int):
        self.n = int(n)
        self._ops: list[tuple] = []
        self._params: list[float] = []

    # -- construction ---------------------------------------------------
    def _add(self, kind, target, width=0, controls=None, params=()):
        mask, val = _ctrl_bits(controls)
        off = len(self._params)
        self._params.extend(float(p) for p in params)
        self._ops.append((kind, int(target), int(width), 0, mask, val, off if params else 0))
        return self

    def _add_masked(self, kind, target, width, mask, val, params=()):
        off = len(self._params)
        self._params.extend(float(p) for p in params)
        self._ops.append((kind, int(target), int(width), 0, int(mask), int(val), off if params else 0))
        return self

    def u(self, t, mat, controls=None):
        m = np.asarray(mat, dtype=np.complex128).reshape(2, 2)
        flat = []
        for z in m.reshape(-1):
            flat += [z.real, z.imag]
        return self._add(U, t, 0, controls, flat)

    def h(self, t, controls=None):
        return self.u(t, _H, controls)

    def x(self, t, controls=None):
        return self._add(X, t, 0, controls)

    def ry(self, t, theta, controls=None):
        return self._add(RY, t, 0, controls, (theta,))

    def phase(self, t, theta, controls=None):
        return self._add(PHASE, t, 0, controls, (theta,))

    def s(self, t, controls=None):
        return self.phase(t, np.pi / 2, controls)

    def sdg(self, t, controls=None):
        return self.phase(t, -np.pi / 2, controls)

    def inc(self, base, width, controls=None):
        return self._add(INC, base, width, controls)

    def dec(self, base, width, controls=None):
        return self._add(DEC, base, width, controls)

    def swap(self, a, b, controls=None):
        return self._add(SWAP, a, b, controls)

    def projphase(self, signal, mask, val, theta):
        return self._add_masked(PROJPHASE, signal, 0, mask, val, (theta,))

    def append_op(self, rec, params):
        """Append one record (kind, target, width, flags, mask, val) with its params."""
        kind, target, width, _flags, mask, val = rec[:6]
        return self._add_masked(kind, target, width, mask, val, params)

    def extend(self, other: "Circuit"):
        if other.n > self.n:
            raise ValueError("cannot extend with a wider circuit")
        for rec, prm in other.iter_ops():
            self.append_op(rec, prm)
        return self

    # -- inspection -----------------------------------------------------
    def __len__(self):
        return len(self._ops)

    def iter_ops(self):
        nparam = {U: 8, RY: 1, PHASE: 1, PROJPHASE: 1}
        for rec in self._ops:
            k = rec[0]
            cnt = nparam.get(k, 0)
            yield rec, self._params[rec[6]: rec[6] + cnt]

    def arrays(self):
        ops = np.array(self._ops, dtype=OP_DTYPE) if self._ops else np.zeros(0, OP_DTYPE)
        params = np.array(self._params if self._params else [0.0], dtype=np.float64)
        return ops, params

    def counts(self):
        out = {}
        for rec in self._ops:
            out[KIND_NAMES[rec[0]]] = out.get(KIND_NAMES[rec[0]], 0) + 1
        return out

    def dagger(self) -> "Circuit":
        """The inverse circuit: reversed order, each op inverted."""
        inv = Circuit(self.n)
        for rec, prm in reversed(list(self.iter_ops())):
            kind = rec[0]
            if kind == U:
                m = np.array(prm[0::2]) + 1j * np.array(prm[1::2])
                m = m.reshape(2, 2).conj().T
                flat = []
                for z in m.reshape(-1):
                    flat += [z.real, z.imag]
                inv.append_op(rec, flat)
            elif kind in (RY, PHASE, PROJPHASE):
                inv.append_op(rec, [-prm[0]])
            elif kind == INC:
                inv.append_op((DEC,) + tuple(rec[1:]), [])
            elif kind == DEC:
                inv.append_op((INC,) + tuple(rec[1:]), [])
            else:
                inv.append_op(rec, prm)
        return inv


def from_arrays(n, ops, params) -> Circuit:
    c = Circuit(n)
    nparam = {U: 8, RY: 1, PHASE: 1, PROJPHASE: 1}
    for r in ops:
        k = int(r["kind"])
        cnt = nparam.get(k, 0)
        off = int(r["param"])
        c.append_op((k, int(r["target"]), int(r["width"]), 0, int(r["ctrl_mask"]), int(r["ctrl_val"])),
                    list(params[off: off + cnt]))
    return c

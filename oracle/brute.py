"""Dense-unitary brute force for a handful of qubits (NumPy).

TEST INFRASTRUCTURE ONLY.  Each op becomes its full 2^n x 2^n matrix, built
from textbook identities rather than from index arithmetic:

* a controlled single-qubit gate is  P_c (x) M + (I - P_c) (x) I, with P_c the
  tensor product of |v><v| on the control qubits (Kronecker products, qubit 0
  the rightmost factor);
* R_Y(theta) is the matrix exponential of -i theta Y / 2 (scipy.linalg.expm);
* a cyclic +1 on a w-qubit register is the standard ripple of multi-controlled
  X gates, most significant bit first: X on bit j controlled by all lower
  register bits being 1; -1 is its conjugate transpose;
* SWAP is three CNOTs;
* the QSVT projector phase is its three-gate form MCX . exp(i theta Z) . MCX.
"""
from __future__ import annotations

from functools import reduce

import numpy as np
import scipy.linalg

I2 = np.eye(2, dtype=np.complex128)
XM = np.array([[0, 1], [1, 0]], dtype=np.complex128)
YM = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
P0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)
P1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)

KIND_U, KIND_X, KIND_PHASE, KIND_RY, KIND_INC, KIND_DEC, KIND_SWAP, KIND_PROJ = range(8)


def _kron_list(factors_by_qubit):
    # qubit n-1 is the leftmost factor so that index bit j <-> qubit j
    return reduce(np.kron, factors_by_qubit[::-1])


def controlled(n, target, m, ctrl: dict) -> np.ndarray:
    proj = [I2] * n
    for q, v in ctrl.items():
        proj[q] = P1 if v else P0
    full_on = list(proj)
    full_on[target] = m
    P = _kron_list(proj)
    return _kron_list(full_on) + (np.eye(1 << n) - P)


def _ctrl_dict(mask, val, n):
    return {q: (val >> q) & 1 for q in range(n) if (mask >> q) & 1}


def increment(n, base, width, ctrl: dict) -> np.ndarray:
    U = np.eye(1 << n, dtype=np.complex128)
    for j in range(width - 1, -1, -1):
        c = dict(ctrl)
        for l in range(j):
            c[base + l] = 1
        U = controlled(n, base + j, XM, c) @ U
    return U


def op_matrix(n, rec, prm) -> np.ndarray:
    kind = int(rec["kind"])
    t = int(rec["target"])
    ctrl = _ctrl_dict(int(rec["ctrl_mask"]), int(rec["ctrl_val"]), n)
    if kind == KIND_U:
        m = (np.array(prm[0::2]) + 1j * np.array(prm[1::2])).reshape(2, 2)
        return controlled(n, t, m, ctrl)
    if kind == KIND_X:
        return controlled(n, t, XM, ctrl)
    if kind == KIND_PHASE:
        return controlled(n, t, np.diag([1.0, np.exp(1j * prm[0])]), ctrl)
    if kind == KIND_RY:
        return controlled(n, t, scipy.linalg.expm(-0.5j * prm[0] * YM), ctrl)
    if kind == KIND_INC:
        return increment(n, t, int(rec["width"]), ctrl)
    if kind == KIND_DEC:
        return increment(n, t, int(rec["width"]), ctrl).conj().T
    if kind == KIND_SWAP:
        a, b = t, int(rec["width"])
        cx_ba = dict(ctrl)
        cx_ba[b] = 1
        # with outer controls held fixed, CX(a->b) CX(b->a) CX(a->b) is a controlled SWAP
        A = controlled(n, b, XM, {a: 1})
        B = controlled(n, a, XM, cx_ba)
        return A @ B @ A
    if kind == KIND_PROJ:
        mcx = controlled(n, t, XM, ctrl)
        z = controlled(n, t, np.diag([np.exp(1j * prm[0]), np.exp(-1j * prm[0])]), {})
        return mcx @ z @ mcx
    raise ValueError(kind)


def unitary(circuit) -> np.ndarray:
    ops, params = circuit.arrays()
    n = circuit.n
    nparam = {KIND_U: 8, KIND_RY: 1, KIND_PHASE: 1, KIND_PROJ: 1}
    U = np.eye(1 << n, dtype=np.complex128)
    for rec in ops:
        off = int(rec["param"])
        prm = list(params[off: off + nparam.get(int(rec["kind"]), 0)])
        U = op_matrix(n, rec, prm) @ U
    return U

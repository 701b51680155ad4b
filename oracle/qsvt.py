"""Quantum signal processing and the singular-value transform, evaluated
classically (NumPy, FP64).

TEST INFRASTRUCTURE ONLY.  Definitions (Sec. II.D.5 and the QSVT literature it
cites):

* QSP in the W_x convention: for phases phi_0..phi_d,
      U(x) = e^{i phi_0 Z} W(x) e^{i phi_1 Z} W(x) ... W(x) e^{i phi_d Z},
      W(x) = [[x, i sqrt(1-x^2)], [i sqrt(1-x^2), x]],
  and p(x) = <0|U(x)|0>.  Evaluated here by plain 2x2 matrix products.
* The singular-value transform of an odd polynomial f of a matrix M with SVD
  M = sum_i s_i |w_i><v_i| is f^{SV}(M) = sum_i f(s_i) |w_i><v_i|.
* A block encoding's encoded matrix is lambda <0_anc| U |0_anc>.
"""
from __future__ import annotations

import numpy as np


def qsp_unitary(phases, x: float) -> np.ndarray:
    """The 2x2 QSP product U(x) for one real x in [-1, 1]."""
    s = np.sqrt(max(0.0, 1.0 - x * x))
    Wx = np.array([[x, 1j * s], [1j * s, x]], dtype=np.complex128)
    def rz(p):
        return np.diag([np.exp(1j * p), np.exp(-1j * p)])
    Um = rz(phases[0])
    for p in phases[1:]:
        Um = Um @ Wx @ rz(p)
    return Um


def qsp_poly(phases, xs) -> np.ndarray:
    """p(x) = <0|U(x)|0> for every x in xs (complex)."""
    return np.array([qsp_unitary(phases, float(x))[0, 0] for x in np.atleast_1d(xs)])


def chebyshev_eval(coefs_odd, xs) -> np.ndarray:
    """sum_j c_j T_{2j+1}(x), with T_n(x) = cos(n arccos x), for |x| <= 1."""
    xs = np.atleast_1d(np.asarray(xs, float))
    th = np.arccos(np.clip(xs, -1.0, 1.0))
    out = np.zeros_like(xs)
    for j, c in enumerate(coefs_odd):
        out += c * np.cos((2 * j + 1) * th)
    return out


def sv_transform(M: np.ndarray, f) -> np.ndarray:
    """f^{SV}(M) = sum_i f(s_i) |w_i><v_i| for an odd function f (vectorised)."""
    Wm, s, Vh = np.linalg.svd(M)
    return (Wm * f(s)[None, :]) @ Vh


def project_block(U: np.ndarray, n: int, anc_qubits, sys_qubits) -> np.ndarray:
    """<0_anc| U |0_anc> as a matrix on the system qubits (dense U on n qubits,
    qubit j = bit j of the index; system index bits in the order sys_qubits)."""
    idx = []
    for s in range(1 << len(sys_qubits)):
        i = 0
        for j, q in enumerate(sys_qubits):
            if (s >> j) & 1:
                i |= 1 << q
        idx.append(i)
    idx = np.array(idx)
    return U[np.ix_(idx, idx)]

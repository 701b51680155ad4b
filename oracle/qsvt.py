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

import ctypes

import numpy as np
import scipy.fft as sfft


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
    Wm, s, Vh = np.linalg.svd(M, full_matrices=False)
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


def qsp_poly_batch(phases, xs) -> np.ndarray:
    """p(x) for an array of x: the same 2x2 products as qsp_unitary, carried
    for all x at once (the first row of the running product)."""
    xs = np.asarray(xs, float)
    s = np.sqrt(np.clip(1.0 - xs * xs, 0.0, None))
    row0 = np.full(xs.shape, np.exp(1j * phases[0]), dtype=np.complex128)
    row1 = np.zeros(xs.shape, dtype=np.complex128)
    for p in phases[1:]:
        # [row0, row1] @ [[x, i s], [i s, x]] @ diag(e^{ip}, e^{-ip})
        n0 = (row0 * xs + row1 * 1j * s) * np.exp(1j * p)
        n1 = (row0 * 1j * s + row1 * xs) * np.exp(-1j * p)
        row0, row1 = n0, n1
    return row0


def qsp_poly_points(phases, xs) -> np.ndarray:
    """p(x) for an array of x by the same left-to-right 2x2 products as
    qsp_poly_batch, in the oracle's C library (points in parallel)."""
    from . import statevector as _sv
    ph = np.ascontiguousarray(phases, dtype=np.float64)
    xs = np.ascontiguousarray(xs, dtype=np.float64)
    out = np.empty(len(xs), dtype=np.complex128)
    dp = ctypes.POINTER(ctypes.c_double)
    _sv.lib().oracle_qsp_poly(ph.ctypes.data_as(dp), len(ph) - 1, xs.ctypes.data_as(dp), len(xs),
                              out.ctypes.data_as(dp))
    return out


def odd_chebyshev_of_qsp(phases) -> np.ndarray:
    """Coefficients of T_1, T_3, ..., T_d of Re p for odd d = len(phases) - 1,
    by interpolation at the d + 1 Gauss-Chebyshev nodes x_k = cos theta_k:
    c_n = (2 / N) sum_k Re p(x_k) cos(n theta_k), N = d + 1, which is a DCT-II
    of the node values (the library transform keeps large d in memory)."""
    d = len(phases) - 1
    N = d + 1
    x = np.cos(np.pi * (2 * np.arange(N) + 1) / (2 * N))
    g = qsp_poly_points(phases, x).real
    return (sfft.dct(g, type=2) / N)[1:d + 1:2]


def odd_sv_apply(matvec, rmatvec, coefs, b) -> np.ndarray:
    """f^{SV}(M) b for f = sum_j coefs_j T_{2j+1}, using only products with M
    (matvec) and M^dagger (rmatvec).  For odd n, T_n(s) = s q_n(s^2) with
    q_1 = 1, q_{-1} = 1 and q_{n+2} = (4 s^2 - 2) q_n - q_{n-2}; hence
    f^{SV}(M) b = M sum_j coefs_j q_{2j+1}(M^dagger M) b."""
    def G(v):
        return 4.0 * rmatvec(matvec(v)) - 2.0 * v
    r_prev = np.array(b, dtype=np.complex128)   # q_{-1}
    r = np.array(b, dtype=np.complex128)        # q_1
    acc = coefs[0] * r
    for c in coefs[1:]:
        r_prev, r = r, G(r) - r_prev
        acc = acc + c * r
    return matvec(acc)

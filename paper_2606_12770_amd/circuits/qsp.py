"""QSP phases for the matrix-inversion polynomial of the QSVT solver (host setup,
untimed).

Target (Sec. II.D.5): an odd polynomial f of degree d with f(x) ~ c / x on
[1/kappa, 1] and |f| <= 1/2 on [-1, 1]: the closed-form polynomial of least
maximal relative error (inverse_polynomial), relative error about
2 exp(-d / kappa), and c puts the maximum of |f| at 1/2.

Phases (W_x convention, d + 1 of them, symmetric phi_j = phi_{d-j}):
    p(x) = <0| e^{i phi_0 Z} W(x) e^{i phi_1 Z} ... W(x) e^{i phi_d Z} |0>,
    W(x) = exp(i arccos(x) X),  Re p = f.
They are found by the fixed-point iteration of Dong, Lin, Ni and Wang
("Infinite quantum signal processing", 2022) on the reduced phases
psi = phi - (pi/4)(e_0 + e_d): psi <- psi + (F(psi) - c) / 2, where F maps
reduced phases to the odd Chebyshev coefficients of Re p (in this
convention the Jacobian of F at psi = 0 is -2 I).  The paper cites
the optimisation method of Dong et al. (2021) for the same phases; any phases
that realise f give the same circuit output, and the residual is checked.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft as sfft


def _cheb_nodes(N: int) -> np.ndarray:
    return np.cos(np.pi * (2 * np.arange(N) + 1) / (2 * N))


def _grid_size(d: int) -> int:
    return 1 << max(4, math.ceil(math.log2(4 * (d + 1))))


def odd_chebyshev_coefficients(fun, d: int, N: int | None = None) -> np.ndarray:
    """Coefficients c_j of T_{2j+1}, j = 0..(d-1)/2, of the Chebyshev
    interpolant of fun at N Gauss-Chebyshev nodes (N >= d + 1), by a DCT-II:
    c_n = (2 / N) sum_k fun(x_k) cos(n theta_k), x_k = cos theta_k."""
    if d % 2 == 0:
        raise ValueError("degree must be odd")
    N = N or _grid_size(d)
    y = sfft.dct(fun(_cheb_nodes(N)), type=2) / N
    return y[1:d + 1:2].copy()


def odd_values_on_nodes(coefs: np.ndarray, N: int) -> np.ndarray:
    """sum_j coefs_j T_{2j+1}(x_k) at the N Gauss-Chebyshev nodes x_k (DCT-III)."""
    a = np.zeros(N)
    a[1:2 * len(coefs):2] = coefs
    return sfft.dct(a, type=3) / 2.0


def chebyshev_odd_eval(coefs: np.ndarray, x) -> np.ndarray:
    th = np.arccos(np.clip(np.asarray(x, float), -1.0, 1.0))
    js = np.arange(1, 2 * len(coefs), 2)
    return np.cos(np.multiply.outer(th, js)) @ coefs


def _chebyshev_t_outside(n: int, half_gap: np.ndarray, above: bool) -> np.ndarray:
    """T_n(y) for y = 1 + 2 h (above, h >= 0) or y = 1 - 2 h (inside, 0 <= h <= 1),
    given h, through the half-angle forms arccosh y = 2 asinh(sqrt h) and
    arccos y = 2 asin(sqrt h), which stay accurate for y next to 1."""
    r = np.sqrt(np.maximum(half_gap, 0.0))
    if above:
        return np.cosh(2.0 * n * np.arcsinh(r))
    return np.cos(2.0 * n * np.arcsin(np.minimum(r, 1.0)))


def inverse_polynomial(kappa: float, d: int, peak: float = 0.5):
    """Odd Chebyshev coefficients of the degree-d approximation of c / x on
    [1/kappa, 1].  Returns (coefs, c, max relative error on [1/kappa, 1]).

    The polynomial (Sec. II.D.5 asks for p ~ 1/x on [1/kappa, 1]; the degree
    bound the paper adopts, Eq. d-star, is the one of the polynomial with the
    least maximal relative error) is, with a = 1/kappa, n = (d + 1)/2 and
    g(x) = (1 + a^2 - 2 x^2) / (1 - a^2),
        P(x) = (1 - T_n(g(x)) / T_n(g(0))) / x,
    odd and of degree 2n - 1 = d.  On [a, 1], g maps into [-1, 1], so
    |x P(x) - 1| <= 1 / T_n(g(0)) ~ 2 exp(-d / kappa).  Below a, g > 1 and P
    falls under 1/x (singular values under 1/kappa are under-inverted).
    Coefficients come from the values at a Gauss-Chebyshev grid of at least
    16 (d + 1) points (exact for a degree-d polynomial); c scales the grid
    maximum of |P| on [-1, 1] to `peak`."""
    if d % 2 == 0:
        raise ValueError("degree must be odd")
    if kappa <= 1.0:
        raise ValueError("kappa must exceed 1")
    n = (d + 1) // 2
    a = 1.0 / kappa
    N = max(1 << 15, 1 << math.ceil(math.log2(16 * (d + 1))))
    x = _cheb_nodes(N)
    ax = np.abs(x)
    one_m_a2 = (1.0 - a) * (1.0 + a)
    # g - 1 = 2 (a^2 - x^2) / (1 - a^2),  1 - g = 2 (x^2 - a^2) / (1 - a^2),  1 + g = 2 (1 - x^2) / (1 - a^2)
    low = ax < a
    Tg = np.empty(N)
    Tg[low] = _chebyshev_t_outside(n, (a - ax[low]) * (a + ax[low]) / one_m_a2, True)
    mid = ~low & (ax * ax <= 0.5 * (1.0 + a * a))     # g >= 0: angle from the y = 1 end
    Tg[mid] = _chebyshev_t_outside(n, (ax[mid] - a) * (ax[mid] + a) / one_m_a2, False)
    top = ~low & ~mid                                   # g < 0: T_n(-y) = (-1)^n T_n(y), y next to 1
    Tg[top] = (-1.0) ** n * _chebyshev_t_outside(n, (1.0 - ax[top]) * (1.0 + ax[top]) / one_m_a2, False)
    Tg0 = float(_chebyshev_t_outside(n, np.array([a * a / one_m_a2]), True)[0])
    P = (1.0 - Tg / Tg0) / ax * np.sign(x)
    co = (sfft.dct(P, type=2) / N)[1:d + 1:2]
    vals = odd_values_on_nodes(co, N)
    scale = peak / np.max(np.abs(vals))
    inside = x >= a
    err = float(np.max(np.abs(vals[inside] * x[inside] - 1.0)))
    return co * scale, scale, err


def qsp_real_part(phases: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Re <0|U(x)|0> for all x at once (row vector recursion, O(d) per point)."""
    x = np.asarray(x, float)
    s = np.sqrt(np.clip(1.0 - x * x, 0.0, None))
    e0 = np.exp(1j * phases[0])
    r0 = np.full(x.shape, e0, dtype=np.complex128)
    r1 = np.zeros(x.shape, dtype=np.complex128)
    for p in phases[1:]:
        a = x * r0 + 1j * s * r1
        b = 1j * s * r0 + x * r1
        ep = np.exp(1j * p)
        r0 = a * ep
        r1 = b * np.conj(ep)
    return r0.real


def qsp_chebyshev(phases: np.ndarray) -> np.ndarray:
    """Chebyshev coefficients p_0..p_d (complex) of p(x) = <0|U(x)|0>.

    With x = cos theta, W(x) = [[cos, i sin], [i sin, cos]](theta), so every
    factor W e^{i phi_j Z} is a trigonometric polynomial of degree 1 in theta
    and a product of m factors one of degree m.  The product is formed by
    pairwise halving: a segment of degree m is held by its values at 4m
    equispaced theta; two neighbours are resampled to 8m points (FFT, zero
    padding, inverse FFT) and multiplied point by point.  O(d log^2 d) work;
    every intermediate is a unitary matrix, so values stay bounded.  Finally
    p(cos theta) = p_0 + sum_k p_k cos(k theta) gives p_k = 2 c_k (k >= 1)
    from the Fourier coefficients c_k of the (even) function theta -> U_00."""
    phases = np.asarray(phases, float)
    d = len(phases) - 1
    if d < 1:
        return np.array([np.exp(1j * phases[0])])
    S = 4
    th = 2.0 * np.pi * np.arange(S) / S
    c, s = np.cos(th), np.sin(th)
    e = np.exp(1j * phases[1:])[:, None]
    ec = np.conj(e)
    M = np.empty((4, d, S), dtype=np.complex128)      # entries 00, 01, 10, 11
    M[0] = c * e
    M[1] = 1j * s * ec
    M[2] = 1j * s * e
    M[3] = c * ec
    while M.shape[1] > 1:
        if M.shape[1] % 2:
            eye = np.zeros((4, 1, S), dtype=np.complex128)
            eye[0] = eye[3] = 1.0
            M = np.concatenate([M, eye], axis=1)
        F = np.fft.fft(M, axis=-1)
        G = np.zeros(M.shape[:2] + (2 * S,), dtype=np.complex128)
        h = S // 2
        G[..., :h] = F[..., :h]
        G[..., -h:] = F[..., -h:]
        V = np.fft.ifft(G, axis=-1) * 2.0
        A, B = V[:, 0::2], V[:, 1::2]
        M = np.stack([A[0] * B[0] + A[1] * B[2], A[0] * B[1] + A[1] * B[3],
                      A[2] * B[0] + A[3] * B[2], A[2] * B[1] + A[3] * B[3]])
        S *= 2
    four = np.fft.fft(np.exp(1j * phases[0]) * M[0, 0]) / S
    p = 2.0 * four[:d + 1]
    p[0] = four[0]
    return p


def full_phases(reduced: np.ndarray) -> np.ndarray:
    """Symmetric d + 1 phases (d odd) from the reduced ones, with the pi/4 ends."""
    phi = np.concatenate([reduced[::-1], reduced])
    phi[0] += np.pi / 4
    phi[-1] += np.pi / 4
    return phi


def solve_phases(coefs: np.ndarray, tol: float = 1e-13, max_iter: int = 500):
    """Fixed-point iteration for the phases of Re p = sum_j coefs_j T_{2j+1}.
    Returns (phases, iterations, final coefficient residual)."""
    dt = len(coefs)
    psi = np.zeros(dt)
    res = np.inf
    for it in range(1, max_iter + 1):
        F = qsp_chebyshev(full_phases(psi))[1::2].real
        r = F - coefs
        res = float(np.max(np.abs(r)))
        if res < tol:
            return full_phases(psi), it, res
        psi = psi + 0.5 * r
    raise RuntimeError(f"phase iteration did not converge (residual {res:.3e})")


def inversion_phases(kappa: float, d: int):
    """Phases of the degree-d inversion polynomial.  Returns (phases, c, info):
    Re p(x) ~ c / x on [1/kappa, 1]."""
    coefs, c, err = inverse_polynomial(kappa, d)
    phases, it, res = solve_phases(coefs)
    return phases, c, {"approx_rel_err": err, "iterations": it, "residual": res, "coefs": coefs}


def qsvt_degree(kappa: float) -> int:
    """The paper's working degree: d = 10 kappa + 1 (Sec. III.E), made odd."""
    d = int(math.ceil(10.0 * kappa)) + 1
    return d if d % 2 else d + 1

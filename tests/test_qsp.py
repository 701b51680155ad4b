"""QSP phases and the singular-value transform.

Pins of the oracle's QSP evaluation against closed forms (W^d = exp(i d
arccos(x) X), so <0|W^d|0> = T_d(x)), of its recurrence-based transform against
a dense SVD, and of the product's phase solver against the oracle.
"""
import numpy as np
import pytest

from oracle import qsvt as oq
from paper_2606_12770_amd.circuits import qsp


@pytest.mark.parametrize("d", [1, 2, 5, 8])
def test_oracle_qsp_closed_forms(d):
    xs = np.linspace(-1, 1, 23)
    zero = np.zeros(d + 1)
    assert np.max(np.abs(oq.qsp_poly(zero, xs) - np.cos(d * np.arccos(xs)))) < 1e-13
    ends = zero.copy()
    ends[0] = ends[-1] = np.pi / 4
    assert np.max(np.abs(oq.qsp_poly(ends, xs) - 1j * np.cos(d * np.arccos(xs)))) < 1e-13
    rng = np.random.default_rng(d)
    ph = rng.uniform(-np.pi, np.pi, d + 1)
    assert np.max(np.abs(oq.qsp_poly(ph, xs) - oq.qsp_poly_batch(ph, xs))) < 1e-13
    # |p|^2 <= 1 and parity d mod 2
    p = oq.qsp_poly(ph, xs)
    assert np.all(np.abs(p) <= 1 + 1e-13)
    assert np.max(np.abs(oq.qsp_poly(ph, -xs) - (-1) ** d * p)) < 1e-13


def test_oracle_recurrence_transform_matches_svd():
    rng = np.random.default_rng(0)
    M = rng.standard_normal((40, 30)) + 1j * rng.standard_normal((40, 30))
    M /= 1.05 * np.linalg.norm(M, 2)
    ph = rng.uniform(-np.pi, np.pi, 10)
    co = oq.odd_chebyshev_of_qsp(ph)
    b = rng.standard_normal(30) + 1j * rng.standard_normal(30)
    got = oq.odd_sv_apply(lambda v: M @ v, lambda v: M.conj().T @ v, co, b)
    want = oq.sv_transform(M, lambda s: oq.qsp_poly(ph, s).real) @ b
    assert np.max(np.abs(got - want)) < 1e-13
    # the interpolated coefficients reproduce Re p
    xs = np.linspace(-1, 1, 17)
    assert np.max(np.abs(oq.chebyshev_eval(co, xs) - oq.qsp_poly(ph, xs).real)) < 1e-13


@pytest.mark.parametrize("kappa,d", [(4.0, 41), (30.0, 301), (88.0, 881)])
def test_phase_solver_realises_inversion_polynomial(kappa, d):
    phases, c, info = qsp.inversion_phases(kappa, d)
    assert len(phases) == d + 1
    assert np.allclose(phases, phases[::-1])
    xs = np.linspace(-1, 1, 41)
    re = oq.qsp_poly_batch(phases, xs).real
    want = oq.chebyshev_eval(info["coefs"], xs)
    assert np.max(np.abs(re - want)) < 1e-10
    # Re p ~ c / x on [1/kappa, 1] and stays below 1/2 + tolerance everywhere
    xt = np.linspace(1.0 / kappa, 1.0, 501)
    rel = np.abs(oq.qsp_poly_batch(phases, xt).real * xt / c - 1.0)
    assert rel.max() < 5e-3
    dense = np.linspace(-1, 1, 4001)
    assert np.max(np.abs(oq.qsp_poly_batch(phases, dense).real)) < 0.5 + 1e-6


def test_degree_rule():
    assert qsp.qsvt_degree(88.1) == 883
    assert qsp.qsvt_degree(100.0) == 1001
    assert qsp.qsvt_degree(100.0) % 2 == 1


@pytest.mark.parametrize("d", [1, 3, 101, 1001])
def test_fft_product_matches_oracle_matrix_products(d):
    """The pairwise-halving FFT product of the QSP factors against the oracle's
    plain 2x2 products at random points, for random phases."""
    rng = np.random.default_rng(d)
    ph = rng.uniform(-np.pi, np.pi, d + 1)
    p = qsp.qsp_chebyshev(ph)
    xs = rng.uniform(-1.0, 1.0, 7)
    th = np.arccos(xs)
    got = np.cos(np.multiply.outer(th, np.arange(d + 1))) @ p
    want = oq.qsp_poly(ph, xs)
    assert np.max(np.abs(got - want)) < 1e-13 * max(1, np.log2(d + 1))
    # parity of a degree-d QSP polynomial: only T_k with k = d mod 2
    assert np.max(np.abs(p[(d + 1) % 2::2])) < 1e-13


def test_phase_solver_at_the_second_order_paper_degree():
    """kappa = 7100 (the second-order run of Sec. III.E): d = 71001 phases in
    seconds; at 64 sampled points the oracle's plain 2x2 products of those
    phases give the target polynomial and c / x to the approximation error."""
    kappa, d = 7100.0, 71001
    coefs, c, err = qsp.inverse_polynomial(kappa, d)
    assert err < 5e-3
    phases, it, res = qsp.solve_phases(coefs)
    assert len(phases) == d + 1 and res < 1e-12
    rng = np.random.default_rng(0)
    xs = np.concatenate([rng.uniform(1.0 / kappa, 1.0, 60), [1.0 / kappa, 2.0 / kappa, 0.5, 1.0]])
    got = oq.qsp_poly_batch(phases, xs).real
    want = oq.chebyshev_eval(coefs, xs)
    # bound: (d + 1) / 2 coefficients each off by at most the residual
    assert np.max(np.abs(got - want)) < (d + 1) / 2 * res + 1e-11
    assert np.max(np.abs(got * xs / c - 1.0)) < 5e-3

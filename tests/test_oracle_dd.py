"""Pins of the oracle's DD coefficients (Sections 2.4, 2.5) against facts that do
not come from the oracle itself: polynomial reproduction, the textbook
five-point difference, a brute-force cascade of the subdivision, convergence
order on sinusoids and the single-Fourier-mode symbol."""
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import dd, mra, ops


@pytest.mark.parametrize("p", [2, 3])
def test_weights_reproduce_polynomials_exactly(p):
    # degree <= 2p-1 integer polynomials on integer nodes: the canonical
    # prediction at the midpoints is exact (all weights are dyadic).
    rng = np.random.default_rng(p)
    n = 64
    a = np.arange(n, dtype=np.float64)
    for deg in range(2 * p):
        coef = rng.integers(-5, 6, size=deg + 1).astype(np.float64)
        c = np.polyval(coef, a)
        pred = mra.pred_mid(c, 0, p)
        exact = np.polyval(coef, a + 0.5)
        inner = slice(p, n - p)      # stencils that do not wrap
        assert np.array_equal(pred[inner], exact[inner])
    # degree 2p is not reproduced
    c = a ** (2 * p)
    assert not np.allclose(mra.pred_mid(c, 0, p)[p:n - p], (a + 0.5)[p:n - p] ** (2 * p))


def test_weights_textbook_values():
    w2 = dd.midpoint_weights(2)
    assert [w2[o] for o in (-1, 0, 1, 2)] == [Fr(-1, 16), Fr(9, 16), Fr(9, 16), Fr(-1, 16)]
    w3 = dd.midpoint_weights(3)
    assert [w3[o] * 256 for o in (-2, -1, 0, 1, 2, 3)] == [3, -25, 150, 150, -25, 3]


def test_d1_p2_is_textbook_five_point_difference():
    assert dd.d1_coeffs(2) == [Fr(2, 3), Fr(-1, 12)]


@pytest.mark.parametrize("p", [2, 3])
def test_d1_consistency_and_support(p):
    a = dd.d1_coeffs(p)
    assert len(a) == 2 * p - 2
    assert sum(n * an for n, an in enumerate(a, 1)) == Fr(1, 2)
    pp = dd.phi_prime_at_integers(p)
    assert pp[2 * p - 1] == 0 and pp[-(2 * p - 1)] == 0
    assert all(pp[n] == -pp[-n] for n in pp)


@pytest.mark.parametrize("p", [2, 3])
def test_d1_matches_cascade_brute_force(p):
    # phi by 13 rounds of subdivision from an impulse; centred differences of
    # the limit function at the integers approach phi'(n).
    x, v = dd.cascade_phi(p, 13)
    step = x[1] - x[0]
    pp = dd.phi_prime_at_integers(p)
    for n in range(-(2 * p - 1), 2 * p):
        i = int(np.argmin(np.abs(x - n)))
        approx = (v[i + 1] - v[i - 1]) / (2 * step)
        assert abs(approx - float(pp[n])) < 1e-6


def test_d1_p3_exact_values():
    assert dd.d1_coeffs(3) == [Fr(272, 365), Fr(-53, 365), Fr(16, 1095), Fr(1, 2920)]


def test_d2_textbook_and_symbol_negative():
    assert dd.d2_coeffs(2) == [Fr(-5, 2), Fr(4, 3), Fr(-1, 12)]
    assert dd.d2_coeffs(3) == [Fr(-49, 18), Fr(3, 2), Fr(-3, 20), Fr(1, 90)]
    th = np.linspace(1e-3, np.pi, 500)
    for p in (2, 3):
        assert (ops.d2_symbol(th, p) < 0).all()


def _order(errs):
    return np.log2(errs[0] / errs[1])


@pytest.mark.parametrize("p", [2, 3])
def test_convergence_order_on_sinusoids(p):
    e1, e2 = [], []
    for N in (32, 64):
        h = 2 * np.pi / N
        x = np.arange(N) * h
        X, Y = np.meshgrid(x, x)
        f = np.sin(3 * X) * np.cos(2 * Y)
        e1.append(np.abs(ops.d1(f, 1, h, p) - 3 * np.cos(3 * X) * np.cos(2 * Y)).max())
        e2.append(np.abs(ops.lap(f, h, p) + 13 * f).max())
    assert abs(_order(e1) - 2 * p) < 0.15
    assert abs(_order(e2) - 2 * p) < 0.15


@pytest.mark.parametrize("p", [2, 3])
def test_d1_single_mode_symbol(p):
    N, k = 32, 5
    h = 2 * np.pi / N
    x = np.arange(N) * h
    f = np.broadcast_to(np.exp(1j * k * x), (N, N))
    a = [float(c) for c in dd.d1_coeffs(p)]
    sym = 2j * sum(an * np.sin(n * k * h) for n, an in enumerate(a, 1)) / h
    got = ops.d1(f.real, 1, h, p) + 1j * ops.d1(f.imag, 1, h, p)
    assert np.allclose(got, sym * f, atol=1e-12)

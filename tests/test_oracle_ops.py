"""Pins of the oracle's operators: Poisson solve against a dense minimum-norm
solve and a manufactured solution, single-Fourier-mode closed forms of the
velocity / strain / eddy viscosity, circulation conservation, Lamb-Oseen
advection, the dense-matrix twin of F and J, the exactness of the central
difference for the frozen-viscosity JVP, and the paper's own eddy-viscosity
and Reynolds-number arithmetic (Sections 2.3, 3.2.5, 3.3)."""
import math

import numpy as np
import pytest

from oracle import brute, dd, ops
from workloads import Vortex, nu0_from_re, random_field, vorticity_field


def _grid(N):
    h = 2 * np.pi / N
    x = np.arange(N) * h
    X, Y = np.meshgrid(x, x)
    return h, X, Y


@pytest.mark.parametrize("p", [2, 3])
def test_poisson_matches_dense_minimum_norm_solve(p):
    N = 16
    h, X, Y = _grid(N)
    w = random_field(N, 4)
    L = brute.lap_matrix(N, h, p)
    ref = np.linalg.lstsq(L, -w.ravel(), rcond=None)[0]
    got = ops.poisson(w, h, p)
    assert np.abs(got.ravel() - ref).max() < 1e-12 * np.abs(ref).max()
    assert abs(got.mean()) < 1e-14


@pytest.mark.parametrize("p", [2, 3])
def test_poisson_manufactured(p):
    N = 64
    h, X, Y = _grid(N)
    psi = np.sin(3 * X) * np.cos(2 * Y) + 0.3 * np.cos(X + 4 * Y)
    w = -ops.lap(psi, h, p)
    assert np.abs(ops.poisson(w, h, p) - psi).max() < 1e-13


@pytest.mark.parametrize("p", [2, 3])
def test_single_mode_closed_forms(p):
    # psi = sin(x) sin(y): every quantity follows from the discrete symbols
    N = 32
    h, X, Y = _grid(N)
    a = [float(c) for c in dd.d1_coeffs(p)]
    s1 = sum(an * 2 * math.sin(n * h) for n, an in enumerate(a, 1)) / h      # D1 sin = s1 cos
    c2 = [float(c) for c in dd.d2_coeffs(p)]
    s2 = (c2[0] + 2 * sum(c2[n] * math.cos(n * h) for n in range(1, p + 1))) / h ** 2
    psi = np.sin(X) * np.sin(Y)
    w = -2 * s2 * psi
    b = ops.base_fields(w, h, p, ops.Flow(nu0=1e-3, cs=0.17))
    assert np.abs(b["psi"] - psi).max() < 1e-13
    u_ref, v_ref = s1 * np.sin(X) * np.cos(Y), -s1 * np.cos(X) * np.sin(Y)
    assert np.abs(b["u"] - u_ref).max() < 1e-13
    assert np.abs(b["v"] - v_ref).max() < 1e-13
    # S11 = D1x u = s1^2 cos x cos y = -S22, S12 = (D1y u + D1x v)/2 = 0
    S_ref = np.sqrt(2 * 2 * (s1 ** 2 * np.cos(X) * np.cos(Y)) ** 2)
    assert np.abs(ops.strain_rate(b["u"], b["v"], h, p) - S_ref).max() < 1e-12
    assert np.abs(b["nu"] - (1e-3 + (0.17 * h) ** 2 * S_ref)).max() < 1e-14


def test_paper_eddy_viscosity_and_reynolds_arithmetic():
    # eq. (5) with Cs = 0.18, Delta = 12.35 km and |S| = 2.5e-5 1/s gives the
    # quoted nu_tau = 2 (Cs Delta)^2 |S| of about 250 m^2/s (Section 3.2.5);
    # the Smagorinsky momentum diffusivity (Cs Delta)^2 |S| used here is half.
    nu_tau = 2 * (0.18 * 12.35e3) ** 2 * 2.5e-5
    assert abs(nu_tau - 247.0) < 1.0
    fl = ops.Flow(nu0=0.0, cs=0.18, s0=2.5e-5, smag_mode=1)
    u = np.zeros((4, 4))
    assert np.allclose(ops.eddy_viscosity(u, u, 12.35e3, 2, fl), nu_tau / 2)
    # Re = U R / nu: 12.5 m/s * 100 km / 250 = 5000 and 46.8 * 100 km / 125 = 37440
    assert 12.5 * 1e5 / 250 == 5000 and abs(46.8 * 1e5 / 125 - 37440) < 1e-9
    # core-edge speed of the Gaussian vortex ~ omega0 a / 2 (Section 3.2.5:
    # omega0 = 2.5e-4 1/s, a = 100 km, U = 12.5 m/s) and nu0 = Gamma/(2 pi Re)
    g = 2.5e-4 * math.pi * 1e5 ** 2
    assert abs(g / (2 * math.pi * 1e5) - 12.5) < 1e-9
    assert abs(nu0_from_re(5000.0, [Vortex(1.0, 0.3, 0, 0)]) - 1 / (2 * math.pi * 5000)) < 1e-18


@pytest.mark.parametrize("p", [2, 3])
def test_rhs_conserves_circulation(p):
    N = 64
    h, X, Y = _grid(N)
    w = vorticity_field(N, [Vortex(1.0, 0.3, 2.5, 3.1), Vortex(0.8, 0.4, 3.8, 3.2)]) \
        + 0.01 * random_field(N, 3)
    F = ops.rhs(w, h, p, ops.Flow(nu0=1e-3, cs=0.17))
    assert abs(F.sum()) < 1e-12 * np.abs(F).sum()


@pytest.mark.parametrize("p", [2, 3])
def test_lamb_oseen_rhs(p):
    # one axisymmetric vortex: advection vanishes in the continuum, and with
    # constant nu the residual is nu * laplacian(omega) of the Gaussian
    N = 128
    h, X, Y = _grid(N)
    r0, nu = 0.4, 1e-2
    w = vorticity_field(N, [Vortex(1.0, r0, np.pi, np.pi)])
    b = ops.base_fields(w, h, p, ops.Flow(nu0=nu, smag_mode=0))
    adv = ops.advection(b["u"], b["v"], w, h, p)
    r2 = (X - np.pi) ** 2 + (Y - np.pi) ** 2
    lap_exact = w * (4 * r2 / r0 ** 4 - 4 / r0 ** 2)
    F = ops.rhs(w, h, p, ops.Flow(nu0=nu, smag_mode=0), b)
    scale = np.abs(nu * lap_exact).max()
    assert np.abs(adv).max() < 2e-3 * np.abs(b["u"]).max() * np.abs(w).max() / r0
    assert np.abs(F - adv - nu * lap_exact).max() < 1e-3 * scale


@pytest.mark.parametrize("p", [2, 3])
def test_rhs_and_jacobian_match_matrix_twin(p):
    N = 16
    h, X, Y = _grid(N)
    w = vorticity_field(N, [Vortex(1.0, 0.6, 2.8, 3.0), Vortex(0.7, 0.5, 3.8, 3.5)])
    w = w + 0.05 * random_field(N, 8)
    fl = ops.Flow(nu0=2e-3, cs=0.17, mu=0.1)
    Fref, Jm = brute.rhs_matrix_twin(w, h, p, fl.nu0, fl.cs, fl.mu)
    b = ops.base_fields(w, h, p, fl)
    F = ops.rhs(w, h, p, fl, b)
    sc = np.abs(Fref).max()
    assert np.abs(F - Fref).max() < 1e-11 * sc
    v = random_field(N, 21)
    Jv = ops.jvp(v, b, h, p, fl)
    assert np.abs(Jv.ravel() - Jm @ v.ravel()).max() < 1e-11 * np.abs(Jm @ v.ravel()).max()


@pytest.mark.parametrize("p", [2, 3])
def test_jvp_equals_central_difference(p):
    # with nu frozen, F is quadratic in omega: the central difference is exact
    N = 32
    h, X, Y = _grid(N)
    w = vorticity_field(N, [Vortex(1.0, 0.3, 2.5, 3.1), Vortex(1.0, 0.3, 3.7, 3.1)])
    fl = ops.Flow(nu0=1e-3, cs=0.17)
    b = ops.base_fields(w, h, p, fl)
    v = random_field(N, 5, smooth=2)

    def Ffrozen(x):
        bb = ops.base_fields(x, h, p, fl)
        bb["nu"] = b["nu"]
        return ops.rhs(x, h, p, fl, bb)

    for delta in (1e-1, 1.0, 10.0):
        cd = (Ffrozen(w + delta * v) - Ffrozen(w - delta * v)) / (2 * delta)
        Jv = ops.jvp(v, b, h, p, fl)
        assert np.abs(cd - Jv).max() < 1e-10 * np.abs(Jv).max() * max(1.0, delta ** 2)

"""Pins of the oracle's implicit theta-scheme Newton-GMRES step: GMRES against
a direct solve and against the Krylov-space least-squares problem built from
the power basis; the explicit Euler special case (theta = 0); the exact
amplification factor (1 + (1 - theta) z) / (1 - theta z) of every Fourier mode
in the linear case, with the Laplacian symbol typed from the textbook 5-point
rule; Newton's limit against scipy's own nonlinear solver; and the inexact
(frozen eddy viscosity) Newton residual going to zero."""
import math

import numpy as np
import pytest
import scipy.optimize

from oracle import implicit, krylov, mra, ops
from workloads import Vortex, vorticity_field


def test_gmres_full_dimension_is_the_direct_solve():
    rng = np.random.default_rng(7)
    n = 12
    A = np.eye(n) + 0.3 * rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    x, k = implicit.gmres(lambda v: A @ v, b, n)
    assert k == n
    assert np.abs(x - np.linalg.solve(A, b)).max() < 1e-12 * np.abs(x).max()


def test_gmres_minimises_the_residual_over_the_krylov_space():
    rng = np.random.default_rng(8)
    n, m = 30, 6
    A = np.eye(n) + 0.2 * rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    x, k = implicit.gmres(lambda v: A @ v, b, m)
    Kr = np.stack([np.linalg.matrix_power(A, i) @ b for i in range(m)], axis=1)
    Q, _ = np.linalg.qr(Kr)
    y = np.linalg.lstsq(A @ Q, b, rcond=None)[0]
    assert k == m
    assert np.abs(x - Q @ y).max() < 1e-10 * np.abs(x).max()


def test_gmres_zero_rhs():
    x, k = implicit.gmres(lambda v: 2.0 * v, np.zeros(5), 4)
    assert k == 0 and not x.any()


def pair16(eps):
    g = krylov.Grid(J=4, p=2, eps=eps)
    w0 = vorticity_field(16, [Vortex(1.0, 0.7, 2.6, 3.1), Vortex(1.0, 0.7, 3.8, 3.1)])
    return g, krylov.init_state(w0, g)


def test_theta_zero_is_the_explicit_euler_step():
    g, st = pair16(2e-3)
    fl = ops.Flow(nu0=2e-3, cs=0.17)
    dt = 0.05
    got = implicit.theta_step(st, g, fl, 10, dt, 0.0, 1, do_regrid=False).omega_M
    F = krylov.Operator(g, fl, st.index_fine).F(st.omega_M)
    assert np.abs(got - (st.omega_M + dt * F)).max() < 1e-14 * np.abs(st.omega_M).max()


def lam_d2_p2(theta, h):
    # 5-point 4th-order second difference (-1, 16, -30, 16, -1) / 12 on a Fourier mode
    return (-30.0 + 32.0 * np.cos(theta) - 2.0 * np.cos(2 * theta)) / (12.0 * h * h)


@pytest.mark.parametrize("theta", [0.5, 1.0, 0.7])
def test_linear_case_amplification_factor_per_mode(theta):
    N, nu = 32, 0.05
    g = krylov.Grid(J=5, p=2, eps=0.0)
    h = g.h
    x = np.arange(N) * h
    X, Y = np.meshgrid(x, x)
    modes = [(2, 3, 1.0), (1, 0, -0.4), (4, 1, 0.25)]
    w = sum(a * np.sin(kx * X) * np.cos(ky * Y) for kx, ky, a in modes)
    fl = ops.Flow(nu0=nu, smag_mode=0, advect=False)
    st = krylov.init_state(w, g)
    for dt in (0.01, 0.5, 20.0):
        got = mra.prolong(implicit.theta_step(st, g, fl, 10, dt, theta, 1).omega_M, st.index_fine, g.J, g.p)
        ref = 0.0
        for kx, ky, a in modes:
            z = nu * dt * (lam_d2_p2(kx * h, h) + lam_d2_p2(ky * h, h))
            ref = ref + (1.0 + (1.0 - theta) * z) / (1.0 - theta * z) * a * np.sin(kx * X) * np.cos(ky * Y)
        assert np.abs(got - ref).max() < 1e-13


@pytest.mark.parametrize("theta", [0.5, 1.0])
def test_newton_limit_equals_scipy_root(theta):
    """Smagorinsky off: the frozen-viscosity Jacobian is the exact one, Newton
    with full-dimension GMRES converges, and its limit is the root that scipy's
    MINPACK hybrid method finds for G from the same start."""
    g, st = pair16(2e-3)
    fl = ops.Flow(nu0=2e-3, smag_mode=0)
    dt = 0.2
    n = st.omega_M.size
    got = implicit.theta_step(st, g, fl, n, dt, theta, 8, do_regrid=False).omega_M
    sol = scipy.optimize.root(lambda w: implicit.residual(st, w, g, fl, dt, theta), st.omega_M, method="hybr",
                              options={"xtol": 1e-14})
    assert sol.success
    scale = np.abs(st.omega_M).max()
    assert np.abs(got - sol.x).max() < 1e-9 * scale
    assert np.abs(implicit.residual(st, got, g, fl, dt, theta)).max() < 1e-12 * scale
    assert np.abs(got - st.omega_M).max() > 1e-3 * scale        # the step did move


def test_inexact_newton_residual_goes_to_zero():
    """Smagorinsky on: the frozen-viscosity Jacobian is not exact, Newton is
    inexact, and the residual still falls with every iteration."""
    g, st = pair16(2e-3)
    fl = ops.Flow(nu0=2e-3, cs=0.17)
    dt, theta = 0.1, 0.5
    n = st.omega_M.size
    res = []
    for K in (1, 2, 3, 5):
        w = implicit.theta_step(st, g, fl, n, dt, theta, K, do_regrid=False).omega_M
        res.append(np.abs(implicit.residual(st, w, g, fl, dt, theta)).max())
    assert all(b < 0.5 * a for a, b in zip(res, res[1:]))
    assert res[-1] < 1e-9 * np.abs(st.omega_M).max()


def test_crank_nicolson_is_second_order_in_time():
    """One step of the full nonlinear flow at dt and dt/2 (two steps) against a
    fine-step reference: the error falls by about 4 (no regrid: fixed set)."""
    g, st = pair16(0.0)
    fl = ops.Flow(nu0=5e-3, smag_mode=0)
    T = 0.4

    def run(nsub):
        s = st
        for _ in range(nsub):
            s = implicit.theta_step(s, g, fl, 24, T / nsub, 0.5, 3, do_regrid=False)
        return s.omega_M

    ref = run(32)
    e1, e2 = np.abs(run(4) - ref).max(), np.abs(run(8) - ref).max()
    assert 3.5 < e1 / e2 < 4.5

"""Pins of the oracle's exact Jacobian (the eddy viscosity of eq. (5)
linearised too): central differences of F converge to it at second order in
the step while the frozen-viscosity product stays a fixed distance away; it
equals the frozen product when the viscosity does not follow the strain; the
viscosity derivative obeys the Cauchy-Schwarz bound |nu'| <= (Cs h)^2 |S'|;
the exponential Rosenbrock-Euler step becomes second order in time with it
(first order at frozen viscosity); and Newton's method on the theta-scheme
converges quadratically with it."""
import numpy as np
import pytest

from oracle import implicit, krylov, ops
from workloads import Vortex, vorticity_field

N, P = 16, 2


def setup(cs=0.5, smag_mode=2):
    g = krylov.Grid(J=4, p=P, eps=0.0)
    w0 = vorticity_field(N, [Vortex(1.0, 0.7, 2.6, 3.1), Vortex(1.0, 0.7, 3.8, 3.1)])
    fl = ops.Flow(nu0=1e-3, cs=cs, smag_mode=smag_mode)
    return g, w0, fl


def test_central_differences_converge_to_the_exact_product():
    g, w0, fl = setup()
    h = g.h
    base = ops.base_fields(w0, h, P, fl)
    v = np.random.default_rng(3).standard_normal((N, N))
    Je, Jf = ops.jvp_exact(v, base, h, P, fl), ops.jvp(v, base, h, P, fl)
    scale = np.abs(Je).max()
    err = []
    for d in (4e-3, 2e-3, 1e-3):
        fd = (ops.rhs(w0 + d * v, h, P, fl) - ops.rhs(w0 - d * v, h, P, fl)) / (2 * d)
        err.append(np.abs(fd - Je).max() / scale)
        assert np.abs(fd - Jf).max() / scale > 1e-2           # the frozen product is off by O(1) percent
    assert 3.5 < err[0] / err[1] < 4.5 and 3.5 < err[1] / err[2] < 4.5
    assert err[2] < 2e-5


@pytest.mark.parametrize("smag_mode", [0, 1])
def test_exact_equals_frozen_without_local_strain(smag_mode):
    g, w0, fl = setup(smag_mode=smag_mode)
    fl.s0 = 0.3
    base = ops.base_fields(w0, g.h, P, fl)
    v = np.random.default_rng(4).standard_normal((N, N))
    assert np.array_equal(ops.jvp_exact(v, base, g.h, P, fl), ops.jvp(v, base, g.h, P, fl))


def test_viscosity_derivative_bound():
    g, w0, fl = setup()
    h = g.h
    base = ops.base_fields(w0, h, P, fl)
    v = np.random.default_rng(5).standard_normal((N, N))
    uv, vv = ops.velocities(ops.poisson(v, h, P), h, P)
    nup = ops.nu_prime(base, uv, vv, h, P, fl)
    bound = (fl.cs * h) ** 2 * ops.strain_rate(uv, vv, h, P)
    assert np.all(np.abs(nup) <= bound * (1 + 1e-12) + 1e-300)
    assert np.abs(nup).max() > 0.1 * bound.max()


def test_exponential_step_order_in_time():
    """Errors at 2 and 4 substeps of T = 0.4 against 16 exact-Jacobian
    substeps (no regrid): ratio 4 with the exact Jacobian, 2 at frozen
    viscosity."""
    g, w0, fl = setup()
    st = krylov.init_state(w0, g)
    T = 0.4

    def run(ns, exact):
        s = st
        for _ in range(ns):
            s = krylov.step(s, g, fl, 24, T / ns, do_regrid=False, exact=exact)
        return s.omega_M

    ref = run(16, True)
    e_ex = [np.abs(run(k, True) - ref).max() for k in (2, 4)]
    e_fr = [np.abs(run(k, False) - ref).max() for k in (2, 4)]
    assert 3.3 < e_ex[0] / e_ex[1] < 4.7
    assert 1.7 < e_fr[0] / e_fr[1] < 2.5
    assert e_ex[1] < 0.2 * e_fr[1]


def test_newton_converges_quadratically_with_the_exact_jacobian():
    g, w0, fl = setup()
    st = krylov.init_state(w0, g)
    n = 48                                    # GMRES(48) reaches round-off on this system
    dt, theta = 0.2, 0.5
    res = {}
    for exact in (True, False):
        res[exact] = [np.abs(implicit.residual(st, implicit.theta_step(st, g, fl, n, dt, theta, K, do_regrid=False,
                                                                       exact=exact).omega_M,
                                               g, fl, dt, theta)).max() for K in (1, 2, 3)]
    r = res[True]
    assert r[1] < 10 * r[0] ** 2 / np.abs(w0).max() + 1e-13 and r[2] < 1e-12
    assert res[False][2] > 100 * r[2]                        # frozen viscosity: linear convergence

"""Pins of the passive-scalar oracle (Section 3.6): closed forms of the
semi-discrete advection-diffusion equation, conservation of the scalar's
mass, and a dense matrix exponential of the restricted operator.

The finite-difference weights below are typed from the textbook rules (the
4th-order central first difference (8, -1)/12 and the 5-point 4th-order
second difference), not taken from the oracle."""
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import krylov, mra, ops, scalar
import workloads as W


def grid(N):
    h = 2 * math.pi / N
    x = np.arange(N) * h
    return h, x[None, :], x[:, None]


def lam_d2_p2(theta, h):
    # 5-point 4th-order rule (-1, 16, -30, 16, -1) / 12 on a Fourier mode
    return (-30.0 + 32.0 * np.cos(theta) - 2.0 * np.cos(2 * theta)) / (12.0 * h * h)


def s1_d1_p2(theta, h):
    # central difference (8 (f[k+1] - f[k-1]) - (f[k+2] - f[k-2])) / 12 on e^{i k theta}: i * this
    return (16.0 * np.sin(theta) - 2.0 * np.sin(2 * theta)) / (12.0 * h)


def one_step(r0, u, v, kappa, J, p, m, dt, eps=0.0):
    g = krylov.Grid(J=J, p=p, eps=eps)
    st = krylov.init_state(r0, g)
    st = scalar.step(st, g, u, v, kappa, m, dt)
    return mra.prolong(st.omega_M, st.index_fine, J, p), st


def test_pure_diffusion_decays_each_mode_exactly():
    J, N = 5, 32
    h, X, Y = grid(N)
    kappa = 0.03
    modes = [(3, 2, 1.0), (1, -4, 0.5)]
    r0 = sum(a * np.cos(kx * X + ky * Y) for kx, ky, a in modes)
    z = np.zeros((N, N))
    dt = 0.2
    r1, _ = one_step(r0, z, z, np.full((N, N), kappa), J, 2, 20, dt)
    exact = sum(a * math.exp(kappa * dt * (lam_d2_p2(kx * h, h) + lam_d2_p2(ky * h, h))) *
                np.cos(kx * X + ky * Y) for kx, ky, a in modes)
    assert np.abs(r1 - exact).max() < 1e-12


def test_uniform_advection_shifts_phase_by_the_d1_symbol():
    J, N = 5, 32
    h, X, Y = grid(N)
    U, k, dt = 0.7, 3, 0.3
    r0 = np.cos(k * X) + 0 * Y
    z = np.zeros((N, N))
    r1, _ = one_step(r0, np.full((N, N), U), z, z, J, 2, 20, dt)
    exact = np.cos(k * X - U * s1_d1_p2(k * h, h) * dt) + 0 * Y
    assert np.abs(r1 - exact).max() < 1e-12


def test_advection_diffusion_conserves_mass():
    pb = W.plain_pair(J=5)
    h = 2 * math.pi / pb.N
    fl = ops.Flow(nu0=pb.nu0, cs=pb.cs)
    base = ops.base_fields(W.initial_field(pb), h, pb.p, fl)
    r0 = W.vapor_field(pb.N, 3.0) + 0.1 * W.random_field(pb.N, 5, smooth=2)
    r1, _ = one_step(r0, base["u"], base["v"], base["nu"], pb.J, pb.p, 20, 0.05)
    assert abs(scalar.mass(r1, h) - scalar.mass(r0, h)) < 1e-13 * scalar.mass(np.abs(r0), h)
    assert np.abs(r1 - r0).max() > 1e-4        # the scalar did move


@pytest.mark.parametrize("eps", [0.0, 1e-3])
def test_krylov_step_equals_dense_expm_of_restricted_operator(eps):
    """16^2: A = R L Pi built column by column on the active set; the step
    (no regrid) is exp(dt A) r_M, to the Krylov error of m = 24 >= dim."""
    pb = W.plain_pair(J=4)
    h = 2 * math.pi / pb.N
    fl = ops.Flow(nu0=2e-2, cs=pb.cs)
    base = ops.base_fields(W.initial_field(pb), h, pb.p, fl)
    r0 = W.vapor_field(pb.N, 2.0)
    g = krylov.Grid(J=pb.J, p=pb.p, eps=eps)
    st = krylov.init_state(r0, g)
    op = scalar.ScalarOperator(g, st.index_fine, base["u"], base["v"], base["nu"])
    n = st.omega_M.size
    A = np.stack([op.Av(np.eye(n)[i]) for i in range(n)], axis=1)
    dt = 0.1
    ref = scipy.linalg.expm(dt * A) @ st.omega_M
    got = scalar.step(st, g, base["u"], base["v"], base["nu"], min(n, 60), dt, do_regrid=False).omega_M
    assert np.abs(got - ref).max() < 1e-11 * np.abs(ref).max()


def test_coupled_step_uses_the_flow_at_the_start_of_the_step():
    pb = W.plain_pair(J=5)
    gv = krylov.Grid(J=pb.J, p=pb.p, eps=pb.eps)
    gs = krylov.Grid(J=pb.J, p=pb.p, eps=1e-3)
    fl = ops.Flow(nu0=pb.nu0, cs=pb.cs)
    sf = scalar.ScalarFlow(eddy=True)
    w0, r0 = W.initial_field(pb), W.vapor_field(pb.N, 3.0)
    vs, ss = krylov.init_state(w0, gv), krylov.init_state(r0, gs)
    vs2, ss2 = scalar.coupled_step(vs, ss, gv, gs, fl, sf, 10, 10, pb.dt)
    base = ops.base_fields(mra.prolong(vs.omega_M, vs.index_fine, gv.J, gv.p), gv.h, gv.p, fl)
    alone = scalar.step(ss, gs, base["u"], base["v"], base["nu"], 10, pb.dt)
    assert np.array_equal(ss2.omega_M, alone.omega_M)
    assert np.array_equal(vs2.omega_M, krylov.step(vs, gv, fl, 10, pb.dt).omega_M)

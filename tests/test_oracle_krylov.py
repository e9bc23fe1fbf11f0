"""Pins of the oracle's Krylov exponential step: dense-matrix brute force on
tiny grids, the exact linear special case, the 1x1 phi_1 closed form, Arnoldi
orthonormality, Lamb-Oseen viscous decay, circulation conservation, the
energy/enstrophy budget (Section 3.3) and the initial condition's
circulation (Section 3.1)."""
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import krylov, mra, ops
from workloads import Vortex, random_field, vorticity_field


def test_phi1_scalar():
    for z in (-3.0, -0.5, 1e-3, 0.7):
        got = krylov.phi1_e1(np.array([[z]]))[0]
        assert abs(got - math.expm1(z) / z) < 1e-15 * max(1, abs(math.expm1(z) / z))


@pytest.mark.parametrize("eps", [0.0, 2e-3])
def test_step_matches_dense_expm(eps):
    N, p = 16, 2
    g = krylov.Grid(J=4, p=p, eps=eps)
    fl = ops.Flow(nu0=2e-3, cs=0.17)
    w0 = vorticity_field(N, [Vortex(1.0, 0.7, 2.6, 3.1), Vortex(1.0, 0.7, 3.8, 3.1)])
    st = krylov.init_state(w0, g)
    dt = 0.05
    op = krylov.Operator(g, fl, st.index_fine)
    F = op.F(st.omega_M)
    na = F.size
    A = np.stack([op.Av(e) for e in np.eye(na)], axis=1)
    aug = np.zeros((na + 1, na + 1))
    aug[:na, :na] = dt * A
    aug[:na, na] = dt * F
    ref = st.omega_M + scipy.linalg.expm(aug)[:na, na]
    got = krylov.step(st, g, fl, m=min(na, 60), dt=dt, do_regrid=False).omega_M
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


def test_linear_case_exact_decay():
    # no advection, constant nu, eps = 0: F = nu L w, a single symbol value
    # for sin(2x)cos(3y): the Krylov space is one-dimensional and the step is
    # exp(nu lambda dt) for any dt.
    N, p = 32, 2
    g = krylov.Grid(J=5, p=p, eps=0.0)
    h = g.h
    x = np.arange(N) * h
    X, Y = np.meshgrid(x, x)
    w = np.sin(2 * X) * np.cos(3 * Y)
    fl = ops.Flow(nu0=0.05, smag_mode=0, advect=False)
    lam = float(ops.lap_symbol(N, h, p)[3, 2])
    st = krylov.init_state(w, g)
    for dt in (0.01, 1.0, 10.0):
        got = mra.prolong(krylov.step(st, g, fl, 20, dt).omega_M, st.index_fine, g.J, p)
        assert np.abs(got - np.exp(0.05 * lam * dt) * w).max() < 1e-13


def test_arnoldi_orthonormal_hessenberg():
    g = krylov.Grid(J=5, p=2, eps=1e-3)
    fl = ops.Flow(nu0=1e-3, cs=0.17)
    w0 = vorticity_field(32, [Vortex(1.0, 0.4, 2.6, 3.1), Vortex(1.0, 0.4, 3.8, 3.1)])
    st = krylov.init_state(w0, g)
    op = krylov.Operator(g, fl, st.index_fine)
    V, H, m_eff, beta = krylov.arnoldi_mgs(op.Av, op.F(st.omega_M), 20)
    assert m_eff == 20 and beta > 0
    G = V @ V.T
    assert np.abs(G - np.eye(G.shape[0])).max() < 1e-12
    assert np.all(np.tril(H, -2) == 0)
    # Arnoldi relation A V_m = V_{m+1} H
    AV = np.stack([op.Av(v) for v in V[:m_eff]], axis=0)
    assert np.abs(AV.T - V.T @ H).max() < 1e-11 * np.abs(AV).max()


def test_lamb_oseen_decay():
    # Gaussian vortex under constant viscosity decays as
    # Gamma / (pi (r0^2 + 4 nu t)) exp(-r^2 / (r0^2 + 4 nu t))
    N, p, r0, nu = 64, 2, 0.4, 0.01
    g = krylov.Grid(J=6, p=p, eps=0.0)
    fl = ops.Flow(nu0=nu, smag_mode=0)
    vc = Vortex(1.0, r0, np.pi, np.pi)
    st = krylov.run(vorticity_field(N, [vc]), g, fl, m=20, dt=0.1, nsteps=10)
    w = mra.prolong(st.omega_M, st.index_fine, g.J, p)
    rt2 = r0 ** 2 + 4 * nu * st.t
    h = g.h
    x = np.arange(N) * h
    X, Y = np.meshgrid(x, x)
    ref = 1.0 / (np.pi * rt2) * np.exp(-((X - np.pi) ** 2 + (Y - np.pi) ** 2) / rt2)
    assert np.abs(w - ref).max() < 2e-3 * ref.max()
    assert abs(w.max() - ref.max()) < 1e-3 * ref.max()


def test_circulation_conserved_when_all_active():
    g = krylov.Grid(J=5, p=2, eps=0.0)
    fl = ops.Flow(nu0=1e-3, cs=0.17)
    w0 = vorticity_field(32, [Vortex(1.0, 0.4, 2.6, 3.1), Vortex(0.6, 0.3, 3.8, 3.4)])
    st = krylov.run(w0, g, fl, m=15, dt=0.02, nsteps=5)
    w = mra.prolong(st.omega_M, st.index_fine, g.J, 2)
    assert abs(w.sum() - w0.sum()) < 1e-12 * np.abs(w0).sum()


def test_energy_enstrophy_budget():
    # constant nu: dE/dt = -2 nu Z, dZ/dt = -2 nu P up to truncation
    N, p, nu = 64, 2, 5e-3
    g = krylov.Grid(J=6, p=p, eps=0.0)
    fl = ops.Flow(nu0=nu, smag_mode=0)
    w0 = vorticity_field(N, [Vortex(1.0, 0.5, 2.4, 3.1), Vortex(1.0, 0.5, 3.9, 3.1)])
    w0 = w0 - w0.mean()
    dt = 0.005
    st0 = krylov.init_state(w0, g)
    st1 = krylov.step(st0, g, fl, 20, dt)
    st2 = krylov.step(st1, g, fl, 20, dt)
    d = [krylov.diagnostics(mra.prolong(s.omega_M, s.index_fine, g.J, p), g) for s in (st0, st1, st2)]
    dE = (d[2]["energy"] - d[0]["energy"]) / (2 * dt)
    dZ = (d[2]["enstrophy"] - d[0]["enstrophy"]) / (2 * dt)
    assert abs(dE + 2 * nu * d[1]["enstrophy"]) < 0.05 * 2 * nu * d[1]["enstrophy"]
    assert abs(dZ + 2 * nu * d[1]["palinstrophy"]) < 0.05 * 2 * nu * d[1]["palinstrophy"]


def test_initial_condition_circulation():
    N = 256
    vs = [Vortex(1.0, 0.3, np.pi - 0.6, np.pi), Vortex(0.5, 0.25, np.pi + 0.6, np.pi)]
    w = vorticity_field(N, vs)
    h = 2 * np.pi / N
    assert abs(h * h * w.sum() - 1.5) < 1e-12

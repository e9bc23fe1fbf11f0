"""GPU edge cases of the integrators against the FP64 oracle and closed forms:
the happy breakdown of the Arnoldi process (a single Fourier mode without
advection spans a one-dimensional Krylov space; n modes an n-dimensional one)
in the exponential step and in the theta-scheme's GMRES, and the 6-point
(p = 3) instantiations of the exact-Jacobian products and of the
theta-scheme."""
import dataclasses
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import implicit as oi, krylov as ok, mra as om, ops as oo
import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1604_08159_amd as m
    m.lib()
    return m


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, torch.float64)


def lam_d2_p2(theta, h):
    # 5-point 4th-order second difference (-1, 16, -30, 16, -1) / 12 on a Fourier mode
    return (-30.0 + 32.0 * math.cos(theta) - 2.0 * math.cos(2 * theta)) / (12.0 * h * h)


@pytest.mark.parametrize("integ", ["exponential", "theta"])
def test_single_mode_breakdown(M, integ):
    """w = cos(3x): u = 0 and v w depends on x only, so both advection terms
    vanish exactly, F = nu L w, and A v_1 = nu lambda v_1: the basis stops at
    one vector (h_21 at rounding level).  The step is the closed form
    exp(nu lambda dt) or (1 + (1 - theta) z) / (1 - theta z)."""
    J, N, nu, dt, theta = 5, 32, 0.05, 0.4, 0.5
    h = 2 * math.pi / N
    x = np.arange(N) * h
    w0 = np.repeat(np.cos(3 * x)[None, :], N, axis=0)
    s = M.Solve(M.grid_desc(J, 2, 0.0), M.flow_desc(nu, 0.0, smag_mode=0), M.MRA_FP64, 10, dt, _t(w0))
    if integ == "theta":
        s.set_integrator(M.MRA_THETA_NEWTON, theta, 1)     # F is linear: one Newton iteration is exact
    s.step(2)
    dense, diag = s.read()
    z = nu * dt * lam_d2_p2(3 * h, h)
    fac = math.exp(z) if integ == "exponential" else (1 + (1 - theta) * z) / (1 - theta * z)
    got = dense.cpu().numpy()
    assert np.abs(got - fac ** 2 * w0).max() < 1e-13
    g = ok.Grid(J=J, p=2, eps=0.0)
    fl = oo.Flow(nu0=nu, cs=0.0, smag_mode=0)
    st = ok.init_state(w0, g)
    for _ in range(2):
        st = ok.step(st, g, fl, 10, dt) if integ == "exponential" else oi.theta_step(st, g, fl, 10, dt, theta, 1)
    assert st.last_m_eff == 1
    ref = om.prolong(st.omega_M, st.index_fine, J, 2)
    assert np.abs(got - ref).max() < 1e-13
    sc = s.scalars()
    # one F and one product per step: the basis stopped at one vector
    assert sc["evals"] == 2 * (1 + 1) * N * N
    s.close()


@pytest.mark.parametrize("modes", [(3, 5), (3, 5, 7)])
@pytest.mark.parametrize("integ", ["exponential", "theta"])
def test_breakdown_after_several_columns(M, modes, integ):
    """w = sum_k a_k cos(k x): no advection (u = 0 and w depends on x only),
    F = nu L w, and every cos(k x) is an eigenvector of L, so the Krylov space
    of F has the dimension n of the mode set and the Arnoldi process must stop
    after n columns (the delayed second pass finds the breakdown of column
    n - 1 one product later).  Each mode then advances by its own closed
    form, and m_eff = n as in the oracle."""
    J, N, nu, dt, theta = 4, 16, 0.05, 0.4, 0.5      # 16^2: the residual after n columns is ~1e-15 of ||A v||
    h = 2 * math.pi / N
    x = np.arange(N) * h
    amps = [1.0, 0.5, 0.25, 0.125]
    row = sum(a * np.cos(k * x) for a, k in zip(amps, modes))
    w0 = np.repeat(row[None, :], N, axis=0)
    s = M.Solve(M.grid_desc(J, 2, 0.0), M.flow_desc(nu, 0.0, smag_mode=0), M.MRA_FP64, 10, dt, _t(w0))
    if integ == "theta":
        s.set_integrator(M.MRA_THETA_NEWTON, theta, 1)
    s.step(2)
    dense, diag = s.read()
    got = dense.cpu().numpy()
    want_row = np.zeros(N)
    for a, k in zip(amps, modes):
        z = nu * dt * lam_d2_p2(k * h, h)
        fac = math.exp(z) if integ == "exponential" else (1 + (1 - theta) * z) / (1 - theta * z)
        want_row += a * fac ** 2 * np.cos(k * x)
    err = np.abs(got - want_row[None, :]).max()
    print(f"{integ}, modes {modes}: max |GPU - closed form| {err:.2e}")
    assert err < 1e-12
    g = ok.Grid(J=J, p=2, eps=0.0)
    fl = oo.Flow(nu0=nu, cs=0.0, smag_mode=0)
    st = ok.init_state(w0, g)
    for _ in range(2):
        st = ok.step(st, g, fl, 10, dt) if integ == "exponential" else oi.theta_step(st, g, fl, 10, dt, theta, 1)
    assert st.last_m_eff == len(modes)
    ref = om.prolong(st.omega_M, st.index_fine, J, 2)
    assert np.abs(got - ref).max() < 1e-12
    assert s.scalars()["evals"] == 2 * (1 + len(modes)) * N * N
    s.close()


def _three(J=7):
    return dataclasses.replace(W.three_vortex(J=J), noise_amp=0.0)


@pytest.mark.parametrize("integ,exact", [("exponential", True), ("theta", False), ("theta", True)])
def test_p3_integrators_fp64_match_oracle(M, integ, exact):
    pb = _three()
    m_ = 12
    w0 = W.initial_field(pb)
    s = M.Solve(M.grid_desc(pb.J, pb.p, pb.eps), M.flow_desc(pb.nu0, pb.cs), M.MRA_FP64, m_, pb.dt, _t(w0))
    s.set_jacobian(M.MRA_JAC_EXACT if exact else M.MRA_JAC_FROZEN)
    if integ == "theta":
        s.set_integrator(M.MRA_THETA_NEWTON, 1.0, 2)
    print(f"p=3 {integ} exact={exact}: 2 FP64 steps at {pb.N}^2", flush=True)
    s.step(2)
    dense, _ = s.read()
    g = ok.Grid(J=pb.J, p=pb.p, eps=pb.eps)
    fl = oo.Flow(nu0=pb.nu0, cs=pb.cs)
    st = ok.init_state(w0, g)
    for _ in range(2):
        st = (ok.step(st, g, fl, m_, pb.dt, exact=exact) if integ == "exponential"
              else oi.theta_step(st, g, fl, m_, pb.dt, 1.0, 2, exact=exact))
    ref = om.prolong(st.omega_M, st.index_fine, pb.J, pb.p)
    _, mask, _, _ = s.active_set()
    assert np.array_equal(mask.cpu().numpy(), st.mask)
    rel = np.linalg.norm(dense.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"  rel L2 {rel:.3e}")
    assert rel <= 1e-10
    s.close()


def test_p3_exact_jacobian_mixed(M):
    pb = _three()
    m_ = 12
    w0 = W.initial_field(pb)
    s = M.Solve(M.grid_desc(pb.J, pb.p, pb.eps), M.flow_desc(pb.nu0, pb.cs), M.MRA_MIXED, m_, pb.dt, _t(w0))
    s.set_jacobian(M.MRA_JAC_EXACT)
    s.set_integrator(M.MRA_THETA_NEWTON, 0.5, 2)
    s.step(2)
    dense, _ = s.read()
    g = ok.Grid(J=pb.J, p=pb.p, eps=pb.eps)
    fl = oo.Flow(nu0=pb.nu0, cs=pb.cs)
    st = ok.init_state(w0, g)
    for _ in range(2):
        st = oi.theta_step(st, g, fl, m_, pb.dt, 0.5, 2, exact=True)
    ref = om.prolong(st.omega_M, st.index_fine, pb.J, pb.p)
    rel = np.linalg.norm(dense.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"p=3 mixed exact-Jacobian theta step vs oracle: rel L2 {rel:.3e}")
    assert rel <= 1e-5
    s.close()

"""GPU parity of the implicit theta-scheme step (Newton iterations, one
GMRES(m) cycle each) against the FP64 oracle of the same scheme.

Bars: FP64 active sets bit-exact and fields within 1e-10 of the field norm
(the oracle's Arnoldi is modified Gram-Schmidt on I - theta dt J with numpy's
least squares; the GPU's is CGS2 on J with Givens rotations on the shifted
Hessenberg matrix: equal in exact arithmetic); mixed precision within 1e-5;
batched solves bit-identical to the same solves stepped alone.
"""
import ctypes as C

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


def _solve(M, pb, prec, m=None, stream=None):
    w0 = W.initial_field(pb)
    s = M.Solve(M.grid_desc(pb.J, pb.p, pb.eps), M.flow_desc(pb.nu0, pb.cs), prec, m or pb.m, pb.dt, _t(w0),
                stream=stream)
    return s, w0


def _grid_flow(pb):
    return ok.Grid(J=pb.J, p=pb.p, eps=pb.eps), oo.Flow(nu0=pb.nu0, cs=pb.cs)


@pytest.mark.parametrize("theta,K", [(0.5, 1), (0.5, 2), (1.0, 2), (0.0, 1)])
def test_theta_step_fp64_matches_oracle(M, theta, K):
    pb = W.plain_pair()
    s, w0 = _solve(M, pb, M.MRA_FP64)
    s.set_integrator(M.MRA_THETA_NEWTON, theta, K)
    nsteps = 3
    print(f"theta {theta} K {K}: {nsteps} steps of 64^2 FP64", flush=True)
    s.step(nsteps)
    dense, diag = s.read()
    g, fl = _grid_flow(pb)
    st = ok.init_state(w0, g)
    for _ in range(nsteps):
        st = oi.theta_step(st, g, fl, pb.m, pb.dt, theta, K)
    ref = om.prolong(st.omega_M, st.index_fine, pb.J, pb.p)
    _, mask, _, _ = s.active_set()
    assert np.array_equal(mask.cpu().numpy(), st.mask)
    rel = np.linalg.norm(dense.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"  rel L2 {rel:.3e}")
    assert rel <= 1e-10
    assert abs(diag["t"] - nsteps * pb.dt) < 1e-12
    assert int(diag["n_active"]) == st.omega_M.size
    sc = s.scalars()
    assert sc["steps"] == nsteps
    s.close()


def test_theta_step_mixed_error_reported(M):
    pb = W.plain_pair()
    s, w0 = _solve(M, pb, M.MRA_MIXED)
    s.set_integrator(M.MRA_THETA_NEWTON, 0.5, 2)
    s.step(3)
    dense, _ = s.read()
    g, fl = _grid_flow(pb)
    st = ok.init_state(w0, g)
    for _ in range(3):
        st = oi.theta_step(st, g, fl, pb.m, pb.dt, 0.5, 2)
    ref = om.prolong(st.omega_M, st.index_fine, pb.J, pb.p)
    rel = np.linalg.norm(dense.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"mixed theta-step vs oracle after 3 steps: rel L2 {rel:.3e}")
    assert rel <= 1e-5
    s.close()


def test_switching_integrators_mid_run(M):
    """Two exponential steps, two backward-Euler Newton steps, one exponential
    step, on a stream (each switch drops the captured step graph)."""
    pb = W.plain_pair()
    st_ = torch.cuda.Stream(device=DEV)
    with torch.cuda.stream(st_):
        s, w0 = _solve(M, pb, M.MRA_FP64, stream=st_)
    s.step(2, stream=st_)
    s.set_integrator(M.MRA_THETA_NEWTON, 1.0, 2, stream=st_)
    s.step(2, stream=st_)
    s.set_integrator(M.MRA_EXPONENTIAL, stream=st_)
    s.step(1, stream=st_)
    dense, diag = s.read(stream=st_)
    g, fl = _grid_flow(pb)
    st = ok.init_state(w0, g)
    for _ in range(2):
        st = ok.step(st, g, fl, pb.m, pb.dt)
    for _ in range(2):
        st = oi.theta_step(st, g, fl, pb.m, pb.dt, 1.0, 2)
    st = ok.step(st, g, fl, pb.m, pb.dt)
    ref = om.prolong(st.omega_M, st.index_fine, pb.J, pb.p)
    assert np.linalg.norm(dense.cpu().numpy() - ref) <= 1e-10 * np.linalg.norm(ref)
    assert abs(diag["t"] - 5 * pb.dt) < 1e-12
    s.close()


def test_mixed_integrator_batch_equals_alone(M):
    """solve_batch groups solves by integrator; every solve is bit-identical
    to the same solve stepped alone (graphs on a stream)."""
    pbs = [W.fujiwhara_pair(3000 + i, J=6) for i in range(6)]
    cfg = [(M.MRA_THETA_NEWTON, 0.5, 2), (M.MRA_EXPONENTIAL, 0.0, 0), (M.MRA_THETA_NEWTON, 0.5, 2),
           (M.MRA_THETA_NEWTON, 1.0, 1), (M.MRA_EXPONENTIAL, 0.0, 0), (M.MRA_THETA_NEWTON, 0.5, 2)]
    st_ = torch.cuda.Stream(device=DEV)

    def make(pb, c):
        with torch.cuda.stream(st_):
            s, _ = _solve(M, pb, M.MRA_MIXED, m=10, stream=st_)
        s.set_integrator(c[0], c[1], c[2] or 1, stream=st_)
        return s

    alone = []
    for pb, c in zip(pbs, cfg):
        s = make(pb, c)
        s.step(2, stream=st_)
        alone.append(s.read(stream=st_)[0].cpu().numpy())
        s.close()
    solves = [make(pb, c) for pb, c in zip(pbs, cfg)]
    M.solve_batch(solves, [2] * len(solves), stream=st_)
    for s, a in zip(solves, alone):
        assert np.array_equal(s.read(stream=st_)[0].cpu().numpy(), a)
    for s in solves:
        s.close()


def test_set_integrator_errors(M):
    pb = W.plain_pair()
    s, _ = _solve(M, pb, M.MRA_MIXED)
    for bad in [(2, 0.5, 2), (1, -0.1, 2), (1, 1.5, 2), (1, 0.5, 0), (1, 0.5, M.MRA_MAX_NEWTON + 1)]:
        with pytest.raises(M.MraError) as e:
            s.set_integrator(*bad)
        assert e.value.status == 1
    # a passive scalar reads its partner's flow at the start of the step
    r0 = _t(W.vapor_field(pb.N))
    sc = M.ScalarSolve(s, M.grid_desc(pb.J, pb.p, 1e-3), 10, pb.dt, r0)
    with pytest.raises(M.MraError) as e:
        s.set_integrator(M.MRA_THETA_NEWTON, 0.5, 2)
    assert e.value.status == 6
    with pytest.raises(M.MraError) as e:
        sc.set_integrator(M.MRA_THETA_NEWTON, 0.5, 2)
    assert e.value.status == 6
    sc.close()
    s.set_integrator(M.MRA_THETA_NEWTON, 0.5, 2)          # no rider left
    with pytest.raises(M.MraError) as e:
        M.ScalarSolve(s, M.grid_desc(pb.J, pb.p, 1e-3), 10, pb.dt, r0)
    assert e.value.status == 6
    s.close()


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (2, 1e-5)])
def test_theta_fujiwhara512_matches_oracle(M, prec, tol):
    """The benchmark's 512^2 shape (seed 1000), one Crank-Nicolson step with
    two Newton iterations."""
    pb = W.fujiwhara_pair(1000)
    s, w0 = _solve(M, pb, prec)
    s.set_integrator(M.MRA_THETA_NEWTON, 0.5, 2)
    print(f"512^2 theta step, precision {prec}", flush=True)
    s.step(1)
    dense, _ = s.read()
    g, fl = _grid_flow(pb)
    st = oi.theta_step(ok.init_state(w0, g), g, fl, pb.m, pb.dt, 0.5, 2)
    ref = om.prolong(st.omega_M, st.index_fine, pb.J, pb.p)
    rel = np.linalg.norm(dense.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"  rel L2 {rel:.3e}")
    assert rel <= tol
    if prec == 0:
        _, mask, _, _ = s.active_set()
        assert np.array_equal(mask.cpu().numpy(), st.mask)
    s.close()

"""GPU parity of the exact-Jacobian Krylov products (eddy viscosity of eq. (5)
linearised) against the FP64 oracle, for the exponential step and for the
theta-scheme's Newton iterations.

Bars: FP64 active sets bit-exact and fields within 1e-10 of the field norm;
mixed precision within 1e-5; without the local-strain model the exact choice
reproduces the frozen one to rounding (1e-13 in FP64); batches that mix the two choices are
bit-identical to the solves stepped alone.
"""
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


def _solve(M, pb, prec, m=None, smag_mode=2, stream=None):
    w0 = W.initial_field(pb)
    s = M.Solve(M.grid_desc(pb.J, pb.p, pb.eps), M.flow_desc(pb.nu0, pb.cs, smag_mode=smag_mode), prec,
                m or pb.m, pb.dt, _t(w0), stream=stream)
    return s, w0


def _oracle(pb, w0, nsteps, exact, theta=None, K=0, m=None):
    g = ok.Grid(J=pb.J, p=pb.p, eps=pb.eps)
    fl = oo.Flow(nu0=pb.nu0, cs=pb.cs)
    st = ok.init_state(w0, g)
    for _ in range(nsteps):
        if theta is None:
            st = ok.step(st, g, fl, m or pb.m, pb.dt, exact=exact)
        else:
            st = oi.theta_step(st, g, fl, m or pb.m, pb.dt, theta, K, exact=exact)
    return st


@pytest.mark.parametrize("integ", ["exponential", "theta"])
def test_exact_jacobian_fp64_matches_oracle(M, integ):
    pb = W.plain_pair()
    s, w0 = _solve(M, pb, M.MRA_FP64)
    s.set_jacobian(M.MRA_JAC_EXACT)
    theta, K = (None, 0) if integ == "exponential" else (0.5, 2)
    if theta is not None:
        s.set_integrator(M.MRA_THETA_NEWTON, theta, K)
    print(f"exact Jacobian, {integ}: 3 FP64 steps at 64^2", flush=True)
    s.step(3)
    dense, diag = s.read()
    st = _oracle(pb, w0, 3, True, theta, K)
    ref = om.prolong(st.omega_M, st.index_fine, pb.J, pb.p)
    _, mask, _, _ = s.active_set()
    assert np.array_equal(mask.cpu().numpy(), st.mask)
    rel = np.linalg.norm(dense.cpu().numpy() - ref) / np.linalg.norm(ref)
    # the frozen-viscosity run is far from it, so the products did change
    fr = _oracle(pb, w0, 3, False, theta, K)
    rel_fr = np.linalg.norm(om.prolong(fr.omega_M, fr.index_fine, pb.J, pb.p) - ref) / np.linalg.norm(ref)
    print(f"  rel L2 {rel:.3e} (frozen-viscosity run differs by {rel_fr:.3e})")
    assert rel <= 1e-10 and rel_fr > 1e3 * max(rel, 1e-16)
    s.close()


def test_exact_jacobian_mixed_error_reported(M):
    pb = W.plain_pair()
    s, w0 = _solve(M, pb, M.MRA_MIXED)
    s.set_jacobian(M.MRA_JAC_EXACT)
    s.step(3)
    dense, _ = s.read()
    st = _oracle(pb, w0, 3, True)
    ref = om.prolong(st.omega_M, st.index_fine, pb.J, pb.p)
    rel = np.linalg.norm(dense.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"mixed exact-Jacobian step vs oracle after 3 steps: rel L2 {rel:.3e}")
    assert rel <= 1e-5
    s.close()


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (2, 1e-5)])
def test_exact_jacobian_fujiwhara512_matches_oracle(M, prec, tol):
    pb = W.fujiwhara_pair(1000)
    s, w0 = _solve(M, pb, prec)
    s.set_jacobian(M.MRA_JAC_EXACT)
    print(f"512^2 exact-Jacobian step, precision {prec}", flush=True)
    s.step(1)
    dense, _ = s.read()
    st = _oracle(pb, w0, 1, True)
    ref = om.prolong(st.omega_M, st.index_fine, pb.J, pb.p)
    rel = np.linalg.norm(dense.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"  rel L2 {rel:.3e}")
    assert rel <= tol
    s.close()


def test_exact_equals_frozen_without_local_strain(M):
    """Without the local-strain model nu' = 0, so both choices compute the same
    product; they differ only in where D1 is applied to the stream function
    (the frozen product takes psi~ and the stencil, the exact one u_v and v_v
    from the Fourier symbol), so they agree to rounding."""
    pb = W.plain_pair()
    out, masks = [], []
    for jac in (M.MRA_JAC_FROZEN, M.MRA_JAC_EXACT):
        s, _ = _solve(M, pb, M.MRA_FP64, smag_mode=0)
        s.set_jacobian(jac)
        s.step(2)
        out.append(s.read()[0].cpu().numpy())
        masks.append(s.active_set()[1].cpu().numpy())
        s.close()
    assert np.array_equal(masks[0], masks[1])
    rel = np.linalg.norm(out[0] - out[1]) / np.linalg.norm(out[0])
    print(f"frozen vs exact without local strain (FP64): rel L2 {rel:.2e}")
    assert rel <= 1e-13


def test_mixed_jacobian_batch_equals_alone(M):
    pbs = [W.fujiwhara_pair(4000 + i, J=6) for i in range(4)]
    jac = [1, 0, 1, 1]
    st_ = torch.cuda.Stream(device=DEV)

    def make(pb, j):
        with torch.cuda.stream(st_):
            s, _ = _solve(M, pb, M.MRA_MIXED, m=10, stream=st_)
        s.set_jacobian(j)
        return s

    alone = []
    for pb, j in zip(pbs, jac):
        s = make(pb, j)
        s.step(2, stream=st_)
        alone.append(s.read(stream=st_)[0].cpu().numpy())
        s.close()
    solves = [make(pb, j) for pb, j in zip(pbs, jac)]
    M.solve_batch(solves, [2] * len(solves), stream=st_)
    for s, a in zip(solves, alone):
        assert np.array_equal(s.read(stream=st_)[0].cpu().numpy(), a)
    for s in solves:
        s.close()


def test_set_jacobian_errors(M):
    pb = W.plain_pair()
    s, _ = _solve(M, pb, M.MRA_MIXED)
    with pytest.raises(M.MraError) as e:
        s.set_jacobian(2)
    assert e.value.status == 1
    sc = M.ScalarSolve(s, M.grid_desc(pb.J, pb.p, 1e-3), 10, pb.dt, _t(W.vapor_field(pb.N)))
    with pytest.raises(M.MraError) as e:
        sc.set_jacobian(M.MRA_JAC_EXACT)
    assert e.value.status == 6
    s.set_jacobian(M.MRA_JAC_EXACT)          # a scalar may ride on an exact-Jacobian exponential solve
    sc.close()
    s.close()

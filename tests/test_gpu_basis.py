"""The Arnoldi basis the GPU builds is orthonormal over the active set, at
full size and in every precision.  This holds at any size and for every
column: each column's second Gram-Schmidt pass is taken in the next column's
reads of the basis, and the last column's from the partial sums of its own
update, so every stored vector must be orthogonal to rounding level.  The
subdiagonal of the Hessenberg matrix holds the norms taken before
normalisation, so it is positive.  Precision MRA_FP32 stores the basis in
FP32, so its orthonormality is checked at that precision's bar, and its steps
are checked against the FP64 oracle at the mixed-precision bar."""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import krylov as ok, mra as om, ops as oo
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


CASES = {
    "fujiwhara512": lambda: W.fujiwhara_pair(1000),
    "three256_noise": lambda: W.three_vortex(J=8),
    # 1024^2 with noise: nearly every node active, so the prolongation's
    # full-tile path writes and reads the basis in all three precisions
    "three1024_noise": lambda: W.three_vortex(J=10),
}


PRECS = {"fp64": "MRA_FP64", "mixed": "MRA_MIXED", "fp32": "MRA_FP32"}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("prec", sorted(PRECS))
def test_basis_orthonormal(M, case, prec):
    pb = CASES[case]()
    m_ = 30
    w0 = W.initial_field(pb)
    pr = getattr(M, PRECS[prec])
    s = M.Solve(M.grid_desc(pb.J, pb.p, pb.eps), M.flow_desc(pb.nu0, pb.cs), pr, m_, pb.dt,
                torch.from_numpy(w0).to(DEV))
    print(f"{case} {prec}: 2 steps, m = {m_}", flush=True)
    # the regrid at the end of a step changes the active set, so the basis of
    # the second step is indexed by the set the first step left
    s.step(1)
    p = s.ptrs()
    torch.cuda.synchronize()
    na = int(s._arena_view(p.n_active, 1, torch.int64).item())
    s.step(1)
    torch.cuda.synchronize()
    ctrl = s._arena_view(p.control, 16, torch.int32).cpu().numpy()
    k = int(ctrl[0])
    assert ctrl[2] == 0 and k == m_                        # no breakdown at these sizes
    nf = s.N * s.N
    vdt = torch.float32 if prec == "fp32" else torch.float64     # MRA_FP32 stores the basis in FP32
    vs = p.basis_stride
    V = s._arena_view(p.krylov_V, (m_ + 1) * vs, vdt).view(m_ + 1, vs)[:k, :na].cpu().numpy().astype(np.float64)
    G = V @ V.T
    err = np.abs(G - np.eye(k)).max()
    print(f"  N_a {na}, max |V^T V - I| = {err:.2e}")
    # FP64 storage: rounding of the Gram-Schmidt sums; FP32 storage: each entry
    # rounded to 2^-24 relative, so an inner product of unit vectors moves by ~2^-23
    assert err <= (1e-6 if prec == "fp32" else 1e-12)
    H = s._arena_view(p.hessenberg, (m_ + 1) * m_, torch.float64).view(m_ + 1, m_).cpu().numpy()
    sub = np.array([H[j + 1, j] for j in range(k)])
    assert np.all(np.isfinite(H[:k + 1, :k])) and np.all(sub > 0)
    s.close()


def test_basis_orthonormal_largest(M):
    """The largest grid and the largest Krylov dimension (m = 47): the basis
    then spans its whole buffer resource, and columns 32 .. 46 run the
    run-time-column kernels."""
    pb = dataclasses.replace(W.three_vortex(), noise_seed=37440)
    m_ = 47
    s = M.Solve(M.grid_desc(pb.J, pb.p, pb.eps), M.flow_desc(pb.nu0, pb.cs), M.MRA_MIXED, m_, pb.dt,
                torch.from_numpy(W.initial_field(pb)).to(DEV))
    print(f"three-vortex 2048^2 mixed: 2 steps, m = {m_}", flush=True)
    s.step(1)
    p = s.ptrs()
    torch.cuda.synchronize()
    na = int(s._arena_view(p.n_active, 1, torch.int64).item())
    s.step(1)
    torch.cuda.synchronize()
    ctrl = s._arena_view(p.control, 16, torch.int32).cpu().numpy()
    k = int(ctrl[0])
    assert ctrl[2] == 0 and k == m_
    vs = p.basis_stride
    V = s._arena_view(p.krylov_V, (m_ + 1) * vs, torch.float64).view(m_ + 1, vs)[:k, :na].cpu().numpy()
    err = np.abs(V @ V.T - np.eye(k)).max()
    print(f"  N_a {na}, max |V^T V - I| = {err:.2e}")
    assert err <= 1e-12
    H = s._arena_view(p.hessenberg, (m_ + 1) * m_, torch.float64).view(m_ + 1, m_).cpu().numpy()
    assert np.all(np.isfinite(H[:k + 1, :k])) and np.all(np.array([H[j + 1, j] for j in range(k)]) > 0)
    s.close()


def test_fp32_basis_steps_match_oracle(M):
    """Two steps of a 512^2 Fujiwhara solve with the basis stored in FP32
    against the FP64 oracle, at the mixed-precision bar (1e-5 relative L2)."""
    pb = W.fujiwhara_pair(1000)
    w0 = W.initial_field(pb)
    out = {}
    for name in ("MRA_MIXED", "MRA_FP32"):
        s = M.Solve(M.grid_desc(pb.J, pb.p, pb.eps), M.flow_desc(pb.nu0, pb.cs), getattr(M, name), pb.m, pb.dt,
                    torch.from_numpy(w0).to(DEV))
        s.step(2)
        out[name] = s.read()[0].cpu().numpy()
        s.close()
    g = ok.Grid(J=pb.J, p=pb.p, eps=pb.eps)
    fl = oo.Flow(nu0=pb.nu0, cs=pb.cs)
    st = ok.init_state(w0, g)
    for _ in range(2):
        st = ok.step(st, g, fl, pb.m, pb.dt)
    ref = om.prolong(st.omega_M, st.index_fine, pb.J, pb.p)
    for name, d in out.items():
        rel = np.linalg.norm(d - ref) / np.linalg.norm(ref)
        print(f"{name}: 2 steps at 512^2 vs the FP64 oracle, rel L2 {rel:.2e}")
        assert rel <= 1e-5


def test_fp32_basis_theta_step_matches_oracle(M):
    """The theta-scheme's GMRES and Newton updates read the FP32 basis too:
    two Crank-Nicolson steps (two Newton iterations each) against the FP64
    oracle at the mixed-precision bar."""
    from oracle import implicit as oi
    pb = W.plain_pair()
    w0 = W.initial_field(pb)
    s = M.Solve(M.grid_desc(pb.J, pb.p, pb.eps), M.flow_desc(pb.nu0, pb.cs), M.MRA_FP32, pb.m, pb.dt,
                torch.from_numpy(w0).to(DEV))
    s.set_integrator(M.MRA_THETA_NEWTON, 0.5, 2)
    s.step(2)
    dense = s.read()[0].cpu().numpy()
    s.close()
    g = ok.Grid(J=pb.J, p=pb.p, eps=pb.eps)
    fl = oo.Flow(nu0=pb.nu0, cs=pb.cs)
    st = ok.init_state(w0, g)
    for _ in range(2):
        st = oi.theta_step(st, g, fl, pb.m, pb.dt, 0.5, 2)
    ref = om.prolong(st.omega_M, st.index_fine, pb.J, pb.p)
    rel = np.linalg.norm(dense - ref) / np.linalg.norm(ref)
    print(f"MRA_FP32 theta steps vs the FP64 oracle: rel L2 {rel:.2e}")
    assert rel <= 1e-5


def test_fp32_basis_partner_carries_a_scalar(M):
    """A passive scalar takes its partner's precision: coupled to a solve
    whose basis is FP32 it stores its own basis in FP32 too (the arena the
    binding sizes from the partner's precision fits), and it sees the same
    flow to rounding as with a mixed-precision partner."""
    pb = W.plain_pair()
    w0 = torch.from_numpy(W.initial_field(pb)).to(DEV)
    r0 = torch.from_numpy(W.vapor_field(pb.N)).to(DEV)
    out = {}
    for name in ("MRA_MIXED", "MRA_FP32"):
        s = M.Solve(M.grid_desc(pb.J, pb.p, pb.eps), M.flow_desc(pb.nu0, pb.cs), getattr(M, name), pb.m, pb.dt, w0)
        sc = M.ScalarSolve(s, M.grid_desc(pb.J, pb.p, 1e-3), 10, pb.dt, r0)
        for _ in range(3):
            M.solve_batch([s, sc], [1, 1])
        out[name] = sc.read()[0].cpu().numpy()
        assert int(sc.read()[1]["status"]) == 0
        sc.close()
        s.close()
    rel = np.linalg.norm(out["MRA_FP32"] - out["MRA_MIXED"]) / np.linalg.norm(out["MRA_MIXED"])
    print(f"scalar with an FP32-basis partner vs a mixed one, 3 steps: rel L2 {rel:.2e}")
    assert rel <= 1e-6

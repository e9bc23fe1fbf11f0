"""GPU parity on the unequal-strength (Section 3.3) and unequal-size
(Section 3.4) initial-condition families: FP64 steps against the oracle
(active sets bit-exact, fields within 1e-10), and the energy, enstrophy and
circulation the C-ABI reports against the oracle's diagnostics."""
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


@pytest.mark.parametrize("pb", [W.unequal_strength_pair(W.E6_U2_OVER_U1[-1], J=7),
                                W.unequal_strength_pair(W.E6_U2_OVER_U1[2], J=7),
                                W.unequal_size_pair(W.E7_R2_OVER_R1[-1], J=7),
                                W.unequal_size_pair(W.E7_R2_OVER_R1[0], J=7)], ids=lambda p: p.name)
def test_family_fp64_steps_match_oracle(M, pb):
    m_, nsteps = 12, 3
    w0 = W.initial_field(pb)
    s = M.Solve(M.grid_desc(pb.J, pb.p, pb.eps), M.flow_desc(pb.nu0, pb.cs), M.MRA_FP64, m_, pb.dt,
                torch.from_numpy(w0).to(DEV))
    print(f"{pb.name}: {nsteps} FP64 steps at {pb.N}^2", flush=True)
    s.step(nsteps)
    dense, diag = s.read()
    g = ok.Grid(J=pb.J, p=pb.p, eps=pb.eps)
    fl = oo.Flow(nu0=pb.nu0, cs=pb.cs)
    st = ok.run(w0, g, fl, m_, pb.dt, nsteps)
    ref = om.prolong(st.omega_M, st.index_fine, pb.J, pb.p)
    _, mask, _, _ = s.active_set()
    assert np.array_equal(mask.cpu().numpy(), st.mask)
    rel = np.linalg.norm(dense.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"  rel L2 {rel:.3e}")
    assert rel <= 1e-10
    d = ok.diagnostics(ref, g)
    for key in ("energy", "enstrophy", "palinstrophy"):
        assert abs(diag[key] - d[key]) <= 1e-10 * d[key], key
    assert abs(diag["gamma"] - d["gamma"]) <= 1e-10 * abs(d["gamma"])
    s.close()

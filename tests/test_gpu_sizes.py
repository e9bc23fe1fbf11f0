"""GPU steps at the edges of the supported sizes against the FP64 oracle: the
smallest grids (J = j0 + 1: 8^2 for the 4-point rule, 16^2 for the 6-point
rule, where a tile is the whole grid) and the extreme Krylov dimensions m = 1
and m = 47 (columns past 24 run the run-time-column Gram-Schmidt kernels).
Bars: active sets bit-exact, fields within 1e-10 of the field norm."""
import dataclasses

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


def _run(M, pb, m, nsteps, theta=None):
    w0 = W.initial_field(pb)
    s = M.Solve(M.grid_desc(pb.J, pb.p, pb.eps), M.flow_desc(pb.nu0, pb.cs), M.MRA_FP64, m, pb.dt,
                torch.from_numpy(w0).to(DEV))
    if theta is not None:
        s.set_integrator(M.MRA_THETA_NEWTON, theta, 2)
    print(f"{pb.N}^2 p={pb.p} m={m} theta={theta}: {nsteps} FP64 steps", flush=True)
    s.step(nsteps)
    dense, diag = s.read()
    _, mask, _, _ = s.active_set()
    g = ok.Grid(J=pb.J, p=pb.p, eps=pb.eps)
    fl = oo.Flow(nu0=pb.nu0, cs=pb.cs)
    st = ok.init_state(w0, g)
    for _ in range(nsteps):
        st = ok.step(st, g, fl, m, pb.dt) if theta is None else oi.theta_step(st, g, fl, m, pb.dt, theta, 2)
    ref = om.prolong(st.omega_M, st.index_fine, pb.J, pb.p)
    assert np.array_equal(mask.cpu().numpy(), st.mask)
    rel = np.linalg.norm(dense.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"  rel L2 {rel:.3e}, N_a {int(diag['n_active'])}")
    assert rel <= 1e-10
    s.close()


@pytest.mark.parametrize("p,J", [(2, 3), (3, 4)])
@pytest.mark.parametrize("theta", [None, 0.5])
def test_smallest_grids(M, p, J, theta):
    pb = dataclasses.replace(W.plain_pair(J=J), p=p)
    _run(M, pb, 6, 2, theta)


@pytest.mark.parametrize("m", [1, 47])
def test_krylov_dimension_extremes(M, m):
    _run(M, W.plain_pair(), m, 2)

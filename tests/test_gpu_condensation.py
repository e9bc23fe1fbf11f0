"""GPU parity of vapor condensation (Section 2.6's moving interface; the
scalar's residual gains -c f'(r) and its products -c f''(r_n) v) against the
oracle: a shrinking patch in calm air and a patch carried by a vortex pair,
FP64 at 1e-10 (active sets bit-exact) and mixed precision at 1e-5; a
condensing scalar batched with a passive one is bit-identical to both
stepped alone; at 512^2 the patch shrinks by the curvature law
R^2 = R0^2 - 2 kappa t of the gradient flow without over- or undershoot."""
import dataclasses
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import krylov as ok, mra as om, ops as oo, scalar as osc
import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

DV64 = 0.011            # interface width 2 sqrt(2 D_v) = 0.3, three nodes at 64^2
R064 = 1.5


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1604_08159_amd as m
    m.lib()
    return m


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, torch.float64)


def _partner(calm: bool, J: int = 6):
    pb = W.plain_pair(J=J)
    w0 = np.zeros((pb.N, pb.N)) if calm else W.initial_field(pb)
    return dataclasses.replace(pb, dt=0.05), w0


def _gpu(M, pb, w0, r0, prec, kappa0, cond, nsteps, m_s=10, eps_s=1e-3, stream=None):
    v = M.Solve(M.grid_desc(pb.J, pb.p, pb.eps), M.flow_desc(pb.nu0, pb.cs), prec, pb.m, pb.dt, _t(w0),
                stream=stream)
    s = M.ScalarSolve(v, M.grid_desc(pb.J, pb.p, eps_s), m_s, pb.dt, _t(r0), kappa0=kappa0, eddy=False,
                      stream=stream)
    s.set_condensation(cond, stream=stream)
    if nsteps:
        M.solve_batch([v, s], [nsteps, nsteps], stream=stream)
    return v, s


@pytest.mark.parametrize("calm", [True, False])
@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (2, 1e-5)])
def test_condensation_matches_oracle(M, calm, prec, tol):
    pb, w0 = _partner(calm)
    r0 = W.vapor_patch(pb.N, R064, DV64)
    kappa0, nsteps = 2 * DV64, 3
    print(f"condensation 64^2 calm={calm} precision {prec}: {nsteps} steps", flush=True)
    v, s = _gpu(M, pb, w0, r0, prec, kappa0, 1.0, nsteps)
    got, diag = s.read()
    _, mask, _, _ = s.active_set()
    gv = ok.Grid(J=pb.J, p=pb.p, eps=pb.eps)
    gs = ok.Grid(J=pb.J, p=pb.p, eps=1e-3)
    fl = oo.Flow(nu0=pb.nu0, cs=pb.cs)
    sf = osc.ScalarFlow(kappa0=kappa0, eddy=False, cond=1.0)
    _, ss = osc.run(w0, r0, gv, gs, fl, sf, pb.m, 10, pb.dt, nsteps)
    ref = om.prolong(ss.omega_M, ss.index_fine, gs.J, gs.p)
    rel = np.linalg.norm(got.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"  rel L2 {rel:.2e}, N_a {int(diag['n_active'])}")
    if prec == 0:
        assert np.array_equal(mask.cpu().numpy(), ss.mask)
    assert rel <= tol
    # condensation removes vapor: the mass falls
    h = 2 * math.pi / pb.N
    assert h * h * float(got.sum()) < h * h * float(r0.sum())
    s.close()
    v.close()


def test_condensing_and_passive_scalars_batch_bit_identical(M):
    pb, w0 = _partner(False)
    r0 = W.vapor_patch(pb.N, R064, DV64)
    alone = []
    for cond in (1.0, 0.0):
        v, s = _gpu(M, pb, w0, r0, M.MRA_MIXED, 2 * DV64, cond, 3)
        alone.append(s.read()[0].cpu().numpy())
        s.close()
        v.close()
    v = M.Solve(M.grid_desc(pb.J, pb.p, pb.eps), M.flow_desc(pb.nu0, pb.cs), M.MRA_MIXED, pb.m, pb.dt, _t(w0))
    sc = []
    for cond in (1.0, 0.0):
        s = M.ScalarSolve(v, M.grid_desc(pb.J, pb.p, 1e-3), 10, pb.dt, _t(r0), kappa0=2 * DV64, eddy=False)
        s.set_condensation(cond)
        sc.append(s)
    M.solve_batch([v] + sc, [3, 3, 3])
    for s, ref in zip(sc, alone):
        assert np.array_equal(s.read()[0].cpu().numpy(), ref)
        s.close()
    v.close()
    assert not np.array_equal(alone[0], alone[1])


def test_rate_is_checked(M):
    pb, w0 = _partner(True)
    v, s = _gpu(M, pb, w0, W.vapor_patch(pb.N, R064, DV64), M.MRA_MIXED, 2 * DV64, 0.0, 0)
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(M.MraError) as e:
            s.set_condensation(bad)
        assert e.value.status == 1
    with pytest.raises(M.MraError) as e:
        M.ScalarSolve.set_condensation(v, 1.0)          # a vorticity solve has no condensation
    assert e.value.status == 6
    s.close()
    v.close()


def test_patch_shrinks_by_the_curvature_law_512(M):
    """Section 2.6's experiment at 512^2 in calm air: the area A of the patch
    (h^2 sum r) follows R^2 = A / pi = R0^2 - 2 kappa t (the gradient flow's
    sharp-interface law), and r stays within [0, 1] up to 1e-3."""
    pb, w0 = _partner(True, J=9)
    pb = dataclasses.replace(pb, dt=0.1)
    kappa = 2 * W.COND_DV
    r0 = W.vapor_patch(pb.N)
    v, s = _gpu(M, pb, w0, r0, M.MRA_MIXED, kappa, 1.0, 0, m_s=20, eps_s=1e-4)
    h = 2 * math.pi / pb.N
    ts, R2 = [], []
    for k in range(5):
        M.solve_batch([v, s], [50, 50])
        d = s.read()[0].cpu().numpy()
        ts.append(5.0 * (k + 1))
        R2.append(h * h * float(d.sum()) / math.pi)
        assert d.min() >= -1e-3 and d.max() <= 1 + 1e-3
    rate = -np.polyfit(ts[1:], R2[1:], 1)[0]
    print(f"512^2 patch: R^2 {['%.4f' % x for x in R2]} at t = {ts}; -dR^2/dt {rate:.5f} against 2 kappa {2 * kappa:.5f}")
    assert abs(rate - 2 * kappa) <= 0.15 * 2 * kappa
    s.close()
    v.close()

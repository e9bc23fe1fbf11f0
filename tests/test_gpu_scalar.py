"""GPU parity of the passive scalar (Section 3.6) against the oracle: a vapor
field carried by a vorticity solve, stepped together (mra_scalar_init,
solve_batch), FP64 at 1e-10 and mixed precision at 1e-5; mass conservation
with every node active; stepping out of order is refused; batched pairs are
bit-identical to pairs stepped alone."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import krylov as ok, mra as om, ops as oo, scalar as osc
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


def make_pair(M, pb, prec, eps_s, m_s=12, eddy=True, kappa0=0.0, stream=None, sharp=4.0):
    v = M.Solve(M.grid_desc(pb.J, pb.p, pb.eps), M.flow_desc(pb.nu0, pb.cs), prec, pb.m, pb.dt,
                _t(W.initial_field(pb)), stream=stream)
    s = M.ScalarSolve(v, M.grid_desc(pb.J, pb.p, eps_s), m_s, pb.dt, _t(W.vapor_field(pb.N, sharp)),
                      kappa0=kappa0, eddy=eddy, stream=stream)
    return v, s


def oracle_pair(pb, eps_s, nsteps, m_s=12, eddy=True, kappa0=0.0, sharp=4.0):
    gv = ok.Grid(J=pb.J, p=pb.p, eps=pb.eps)
    gs = ok.Grid(J=pb.J, p=pb.p, eps=eps_s)
    fl = oo.Flow(nu0=pb.nu0, cs=pb.cs)
    sf = osc.ScalarFlow(kappa0=kappa0, eddy=eddy)
    vs, ss = osc.run(W.initial_field(pb), W.vapor_field(pb.N, sharp), gv, gs, fl, sf, pb.m, m_s, pb.dt, nsteps)
    return vs, ss, gs


@pytest.mark.parametrize("graph", [False, True])
def test_scalar_fp64_matches_oracle(M, graph):
    pb = W.plain_pair()
    st = torch.cuda.Stream(device=DEV) if graph else None
    ctx = torch.cuda.stream(st) if graph else torch.cuda.stream(torch.cuda.current_stream())
    with ctx:
        v, s = make_pair(M, pb, M.MRA_FP64, 1e-3, stream=st)
    M.solve_batch([v, s], [3, 3], stream=st)
    got, diag = s.read(stream=st)
    _, ss, gs = oracle_pair(pb, 1e-3, 3)
    ref = om.prolong(ss.omega_M, ss.index_fine, gs.J, gs.p)
    rel = np.linalg.norm(got.cpu().numpy() - ref) / np.linalg.norm(ref)
    _, mask, _, _ = s.active_set()
    print(f"scalar FP64 (graph={graph}), 3 steps: rel L2 {rel:.2e}, N_a {ss.omega_M.size}")
    assert rel <= 1e-10
    assert np.array_equal(mask.cpu().numpy(), ss.mask)
    assert diag["status"] == 0
    s.close()
    v.close()


def test_scalar_mixed_matches_oracle(M):
    pb = W.fujiwhara_pair(1000, J=7)
    v, s = make_pair(M, pb, M.MRA_MIXED, 1e-4, m_s=10)
    M.solve_batch([v, s], [2, 2])
    got, _ = s.read()
    _, ss, gs = oracle_pair(pb, 1e-4, 2, m_s=10)
    ref = om.prolong(ss.omega_M, ss.index_fine, gs.J, gs.p)
    rel = np.linalg.norm(got.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"scalar mixed 128^2, 2 steps: rel L2 {rel:.2e}")
    assert rel <= 1e-5
    s.close()
    v.close()


def test_scalar_constant_kappa_and_mass(M):
    """eps = 0 (every node active, regrid exact): the mass h^2 sum(r) is kept."""
    pb = W.plain_pair()
    v, s = make_pair(M, pb, M.MRA_FP64, 0.0, eddy=False, kappa0=2e-3)
    r0, d0 = s.read()
    M.solve_batch([v, s], [4, 4])
    r4, d4 = s.read()
    _, ss, gs = oracle_pair(pb, 0.0, 4, eddy=False, kappa0=2e-3)
    ref = om.prolong(ss.omega_M, ss.index_fine, gs.J, gs.p)
    h = 2 * math.pi / pb.N
    assert np.abs(r4.cpu().numpy() - ref).max() <= 1e-10 * np.abs(ref).max()
    m0, m4 = h * h * float(r0.sum()), h * h * float(r4.sum())
    assert abs(m4 - m0) <= 1e-12 * abs(m0)
    assert abs(d4["gamma"] - m4) <= 1e-12 * abs(m0)
    s.close()
    v.close()


def test_scalar_step_order_is_enforced(M):
    pb = W.plain_pair()
    v, s = make_pair(M, pb, M.MRA_FP64, 1e-3)
    with pytest.raises(M.MraError):
        s.step(1)                      # the partner has not stepped
    v.step(1)
    s.step(1)                          # now in order
    with pytest.raises(M.MraError):
        s.step(1)                      # partner must step again first
    with pytest.raises(M.MraError):
        v.step(1); s.step(2)           # one scalar step per partner step
    s.close()
    v.close()


def test_batched_pairs_equal_pairs_alone(M):
    pbs = [W.plain_pair(), W.fujiwhara_pair(1003, J=6), W.fujiwhara_pair(1004, J=6)]
    st = torch.cuda.Stream(device=DEV)
    alone = []
    for pb in pbs:
        with torch.cuda.stream(st):
            v, s = make_pair(M, pb, M.MRA_MIXED, 1e-3, stream=st)
        M.solve_batch([v, s], [2, 2], stream=st)
        alone.append(s.read(stream=st)[0].cpu().numpy())
        s.close()
        v.close()
    pairs = []
    with torch.cuda.stream(st):
        for pb in pbs:
            pairs.append(make_pair(M, pb, M.MRA_MIXED, 1e-3, stream=st))
    handles = [x for pr in pairs for x in pr]
    M.solve_batch(handles, [2] * len(handles), stream=st)
    for (v, s), a in zip(pairs, alone):
        assert np.array_equal(s.read(stream=st)[0].cpu().numpy(), a)
    for v, s in pairs:
        s.close()
        v.close()

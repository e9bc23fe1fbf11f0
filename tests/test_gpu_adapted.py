"""GPU parity of the level-adapted evaluation (collocation_rhs_adapted and
solves with MRA_EVAL_ADAPTED) against the oracle's adapted mode
(oracle/adapted.py) on the same seeded inputs.

Bars: FP64 within 1e-10 of the scale; with FP32 bulk fields the residual
(FP64) within 1e-10 and the product within the stated 2e-5; masks and index
lists of adapted FP64 steps bit-exact."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import adapted as ad, krylov as ok, mra as om, ops as oo
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


def _t(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


def _field(N, seed, noise=1e-5):
    vs = [W.Vortex(1.0, 0.4, 2.6, 3.1), W.Vortex(0.8, 0.3, 3.9, 3.3)]
    return W.vorticity_field(N, vs) + noise * W.random_field(N, seed)


def _gpu(M, fn, g, f, prec, mask, fi, omega, v=None):
    n = fi.size
    out = torch.empty(n, dtype=torch.float64, device=DEV)
    fn(g, f, prec, _t(mask, torch.uint8), _t(fi, torch.int32), _t(np.array([n]), torch.int64), _t(omega),
       None if v is None else _t(v), out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("p,J,eps", [(2, 6, 1e-3), (2, 8, 1e-4), (3, 7, 1e-3), (3, 8, 1e-4), (2, 5, 3e-2)])
@pytest.mark.parametrize("prec", [0, 2])
def test_adapted_rhs_and_jvp_match_oracle(M, p, J, eps, prec):
    N = 1 << J
    h = 2 * math.pi / N
    u = _field(N, J)
    pk = om.forward(u, J, p)
    mask, ip, fi = om.threshold(pk, u, eps, J, p)
    omega = u.ravel()[fi]
    if prec != M.MRA_FP64:
        omega = omega.astype(np.float32).astype(np.float64)
    fl = oo.Flow(nu0=1e-3, cs=0.17, mu=0.02)
    g, gf = M.grid_desc(J, p, eps), M.flow_desc(1e-3, 0.17, 0.0, 0.02)
    wt = om.prolong(omega, fi, J, p)
    base = oo.base_fields(wt, h, p, fl)
    lam = ad.local_level(fi, J, p)
    assert len(set(lam.tolist())) > 1
    F = ad.rhs(wt, base, fi, lam, h, p, fl)
    got = _gpu(M, M.collocation_rhs_adapted, g, gf, prec, mask, fi, omega)
    errF = np.abs(got - F).max() / np.abs(F).max()
    v = W.random_field(N, 31, smooth=1).ravel()[fi]
    if prec != M.MRA_FP64:
        v = v.astype(np.float32).astype(np.float64)
    Jv = ad.jvp(om.prolong(v, fi, J, p), base, fi, lam, h, p, fl)
    gotv = _gpu(M, M.collocation_rhs_adapted, g, gf, prec, mask, fi, omega, v)
    errJ = np.abs(gotv - Jv).max() / np.abs(Jv).max()
    print(f"adapted p={p} J={J} eps={eps:g} prec={prec} N_a={fi.size}: F {errF:.2e}, J v {errJ:.2e}, "
          f"levels {np.bincount(lam)[om.coarsest_level(p):].tolist()}")
    assert errF <= 1e-10
    assert errJ <= (1e-10 if prec == M.MRA_FP64 else 2e-5)


def test_adapted_with_every_node_active_is_dense(M):
    J, p = 7, 2
    N = 1 << J
    u = _field(N, 3, 1e-2)
    pk = om.forward(u, J, p)
    mask, ip, fi = om.threshold(pk, u, 0.0, J, p)
    g, gf = M.grid_desc(J, p, 0.0), M.flow_desc(1e-3, 0.17)
    omega = u.ravel()[fi]
    a = _gpu(M, M.collocation_rhs_adapted, g, gf, M.MRA_FP64, mask, fi, omega)
    d = _gpu(M, M.collocation_rhs, g, gf, M.MRA_FP64, mask, fi, omega)
    assert np.abs(a - d).max() <= 1e-12 * np.abs(d).max()


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (2, 1e-5)])
def test_adapted_steps_match_oracle(M, prec, tol):
    pb = W.fujiwhara_pair(1004, J=7)
    w0 = W.initial_field(pb)
    s = M.Solve(M.grid_desc(pb.J, pb.p, pb.eps), M.flow_desc(pb.nu0, pb.cs), prec, 12, pb.dt, _t(w0))
    s.set_evaluation(M.MRA_EVAL_ADAPTED)
    g = ok.Grid(J=pb.J, p=pb.p, eps=pb.eps)
    fl = oo.Flow(nu0=pb.nu0, cs=pb.cs)
    st = ok.init_state(w0, g)
    for k in range(1, 4):
        s.step(1)
        st = ok.step(st, g, fl, 12, pb.dt, adapted=True)
        dense, diag = s.read()
        ref = om.prolong(st.omega_M, st.index_fine, pb.J, pb.p)
        rel = np.linalg.norm(dense.cpu().numpy() - ref) / np.linalg.norm(ref)
        _, mask, _, _ = s.active_set()
        flips = int((mask.cpu().numpy() != st.mask).sum())
        print(f"adapted step {k}, precision {prec}: rel L2 {rel:.2e}, mask flips {flips}, N_a {st.omega_M.size}")
        assert diag["status"] == 0
        assert rel <= tol
        if prec == M.MRA_FP64:
            assert flips == 0
    s.close()


def test_adapted_batch_equals_alone_and_errors(M):
    pbs = [W.fujiwhara_pair(1010 + i, J=6) for i in range(3)]
    st = torch.cuda.Stream(device=DEV)

    def make(pb, adapted):
        with torch.cuda.stream(st):
            s = M.Solve(M.grid_desc(pb.J, pb.p, pb.eps), M.flow_desc(pb.nu0, pb.cs), M.MRA_MIXED, 10, pb.dt,
                        _t(W.initial_field(pb)), stream=st)
        if adapted:
            s.set_evaluation(M.MRA_EVAL_ADAPTED)
        return s

    alone = []
    for pb in pbs:
        s = make(pb, True)
        s.step(2, stream=st)
        alone.append(s.read(stream=st)[0].cpu().numpy())
        s.close()
    # adapted and dense solves in one call: two groups, one graph per step
    solves = [make(pb, True) for pb in pbs] + [make(pbs[0], False)]
    M.solve_batch(solves, [2] * len(solves), stream=st)
    for s, a in zip(solves, alone):
        assert np.array_equal(s.read(stream=st)[0].cpu().numpy(), a)
    s = solves[0]
    with pytest.raises(M.MraError) as e:
        s.set_integrator(M.MRA_THETA_NEWTON, 0.5, 2, stream=st)
    assert e.value.status == 6
    with pytest.raises(M.MraError) as e:
        s.set_jacobian(M.MRA_JAC_EXACT)
    assert e.value.status == 6
    with pytest.raises(M.MraError) as e:
        s.set_evaluation(7)
    assert e.value.status == 1
    s.set_evaluation(M.MRA_EVAL_DENSE)
    s.set_jacobian(M.MRA_JAC_EXACT)
    with pytest.raises(M.MraError) as e:
        s.set_evaluation(M.MRA_EVAL_ADAPTED)
    assert e.value.status == 6
    for s in solves:
        s.close()

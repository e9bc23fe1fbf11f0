"""GPU parity at the full sizes of the benchmark configurations, in the launch
configuration bench.py times (batched solves, HIP-graph replay on a
non-default stream).

* 512^2 Fujiwhara pair, 4-point DD, eps 1e-4, m = 20: a batch of 24 seeded
  solves in mixed precision, 2 steps; solve 0 against the FP64 oracle.
* 2048^2 three vortices + noise, 6-point DD, eps 1e-4: F and J v at every
  active node against the oracle (mixed precision), and one m = 30 step in
  FP64 and mixed precision against each other (the oracle's own m = 30 steps
  of this shape run at 512^2 and 1024^2 in test_gpu_configs.py).
"""
import math

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


def _t(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


def test_fujiwhara512_batch_matches_oracle(M):
    pbs = [W.fujiwhara_pair(s) for s in range(1000, 1024)]
    stream = torch.cuda.Stream(device=DEV)
    solves = []
    with torch.cuda.stream(stream):
        for pb in pbs:
            solves.append(M.Solve(M.grid_desc(pb.J, pb.p, pb.eps), M.flow_desc(pb.nu0, pb.cs), M.MRA_MIXED,
                                  pb.m, pb.dt, _t(W.initial_field(pb)), stream=stream))
    M.solve_batch(solves, [2] * len(solves), stream=stream)
    stream.synchronize()
    dense, diag = solves[0].read(stream=stream)
    pb = pbs[0]
    g = ok.Grid(J=pb.J, p=pb.p, eps=pb.eps)
    st = ok.init_state(W.initial_field(pb), g)
    for _ in range(2):
        st = ok.step(st, g, oo.Flow(nu0=pb.nu0, cs=pb.cs), pb.m, pb.dt)
    ref = om.prolong(st.omega_M, st.index_fine, pb.J, pb.p)
    rel = np.linalg.norm(dense.cpu().numpy() - ref) / np.linalg.norm(ref)
    _, mask, _, _ = solves[0].active_set()
    flips = int((mask.cpu().numpy() != st.mask).sum())
    d = ok.diagnostics(ref, g)
    print(f"512^2 batch of 24, mixed, 2 steps: rel L2 {rel:.2e}, mask flips {flips} of {st.omega_M.size}, "
          f"dE/E {abs(diag['energy'] - d['energy']) / d['energy']:.2e}")
    assert diag["status"] == 0
    assert rel <= 1e-6
    assert flips <= 1e-3 * st.omega_M.size
    for s in solves:
        s.close()


@pytest.fixture(scope="module")
def three2048():
    pb = W.three_vortex()
    w0 = W.initial_field(pb)
    pk = om.forward(w0, pb.J, pb.p)
    mask, ip, fi = om.threshold(pk, w0, pb.eps, pb.J, pb.p)
    return pb, w0, mask, fi


def test_three2048_rhs_and_jvp_match_oracle(M, three2048):
    """Mixed precision at 2048^2, 6-point DD, every node active: the residual
    (evaluated in FP64 from the FP32-rounded state) and the FP32 product within
    the stated 2e-5 of their scales."""
    pb, w0, mask, fi = three2048
    h = 2 * math.pi / pb.N
    omega = w0.ravel()[fi].astype(np.float32).astype(np.float64)
    fl = oo.Flow(nu0=pb.nu0, cs=pb.cs)
    wt = om.prolong(omega, fi, pb.J, pb.p)
    base = oo.base_fields(wt, h, pb.p, fl)
    F = oo.rhs(wt, h, pb.p, fl, base).ravel()[fi]
    adv = oo.advection(base["u"], base["v"], wt, h, pb.p).ravel()[fi]
    dif = oo.diffusion(base["nu"], wt, h, pb.p).ravel()[fi]
    sc = max(np.abs(F).max(), np.abs(adv).max(), np.abs(dif).max())
    g = M.grid_desc(pb.J, pb.p, pb.eps)
    gf = M.flow_desc(pb.nu0, pb.cs)
    n = fi.size
    mk, fk, nk = _t(mask, torch.uint8), _t(fi, torch.int32), _t(np.array([n]), torch.int64)
    out = torch.empty(n, dtype=torch.float64, device=DEV)
    M.collocation_rhs(g, gf, M.MRA_MIXED, mk, fk, nk, _t(omega), None, out)
    errF = np.abs(out.cpu().numpy() - F).max() / sc
    v = W.random_field(pb.N, 77, smooth=2).ravel()[fi].astype(np.float32).astype(np.float64)
    vt = om.prolong(v, fi, pb.J, pb.p)
    Jv = oo.jvp(vt, base, h, pb.p, fl).ravel()[fi]
    M.collocation_rhs(g, gf, M.MRA_MIXED, mk, fk, nk, _t(omega), _t(v), out)
    errJ = np.abs(out.cpu().numpy() - Jv).max() / np.abs(Jv).max()
    print(f"2048^2 p=3 N_a={n} ({n / pb.N ** 2:.1%} active): F err {errF:.2e}, J v err {errJ:.2e} (bar 2e-5)")
    assert errF <= 2e-5
    assert errJ <= 2e-5


def test_three2048_step_fp64_vs_mixed(M, three2048):
    pb, w0, mask, fi = three2048
    out = {}
    for prec in (M.MRA_FP64, M.MRA_MIXED):
        s = M.Solve(M.grid_desc(pb.J, pb.p, pb.eps), M.flow_desc(pb.nu0, pb.cs), prec, pb.m, pb.dt, _t(w0))
        s.step(1)
        dense, diag = s.read()
        out[prec] = (dense.cpu().numpy(), diag)
        s.close()
    a, da = out[M.MRA_FP64]
    b, db = out[M.MRA_MIXED]
    rel = np.linalg.norm(a - b) / np.linalg.norm(a)
    print(f"2048^2 one m=30 step: FP64 vs mixed rel L2 {rel:.2e}, N_a {da['n_active']:.0f} / {db['n_active']:.0f}")
    assert da["status"] == 0 and db["status"] == 0
    assert rel <= 1e-5
    assert abs(da["energy"] - db["energy"]) <= 1e-6 * da["energy"]

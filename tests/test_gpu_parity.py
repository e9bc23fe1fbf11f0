"""GPU parity: every C-ABI entry point against the FP64 oracle on the same
seeded inputs.

Bars: masks, index lists and FP64 details / prolongations bit-exact (one
rounding per operation on both sides); FP64 fields within 1e-10 of the field
scale; FP32 fields within 2e-5 of the scale; FP32 masks equal outside a
band of |(|d| - tau)| <= 1e-5 tau + 64 * 2^-24 max|u| around the threshold.
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


def _field(N, seed, noise=1e-3):
    vs = [W.Vortex(1.0, 0.4, 2.6, 3.1), W.Vortex(0.8, 0.3, 3.9, 3.3)]
    return W.vorticity_field(N, vs) + noise * W.random_field(N, seed)


def _t(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


def gpu_forward(M, u, J, p, eps, prec):
    N = 1 << J
    dt = M.bulk_dtype(prec)
    g = M.grid_desc(J, p, eps)
    inp = _t(u, dt)
    out = torch.empty(N * N, dtype=dt, device=DEV)
    mask = torch.empty(N * N, dtype=torch.uint8, device=DEV)
    ip = torch.empty(N * N, dtype=torch.int32, device=DEV)
    fi = torch.empty(N * N, dtype=torch.int32, device=DEV)
    na = torch.zeros(1, dtype=torch.int64, device=DEV)
    M.mra_transform(g, prec, M.MRA_FORWARD, inp, out, mask, ip, fi, na)
    torch.cuda.synchronize()
    n = int(na.item())
    return out.cpu().numpy(), mask.cpu().numpy(), ip[:n].cpu().numpy(), fi[:n].cpu().numpy()


CASES = [(2, 3), (2, 4), (2, 5), (2, 7), (3, 4), (3, 5), (3, 7)]


@pytest.mark.parametrize("p,J", CASES)
@pytest.mark.parametrize("eps", [0.0, 1e-3, 1e-1])
def test_forward_threshold_fp64_bitexact(M, p, J, eps):
    N = 1 << J
    u = _field(N, J)
    pk = om.forward(u, J, p)
    mask, ip, fi = om.threshold(pk, u, eps, J, p)
    gpk, gmask, gip, gfi = gpu_forward(M, u, J, p, eps, M.MRA_FP64)
    assert np.array_equal(gpk, pk)
    assert np.array_equal(gmask, mask)
    assert np.array_equal(gip, ip) and np.array_equal(gfi, fi)


@pytest.mark.parametrize("p,J", [(2, 6), (3, 7)])
def test_forward_threshold_fp32(M, p, J):
    N = 1 << J
    u32 = _field(N, 3).astype(np.float32).astype(np.float64)
    pk = om.forward(u32, J, p)
    eps = 1e-3
    mask, ip, fi = om.threshold(pk, u32, eps, J, p)
    gpk, gmask, _, _ = gpu_forward(M, u32, J, p, eps, M.MRA_FP32)
    umax = np.abs(u32).max()
    assert np.abs(gpk - pk).max() <= 64 * 2.0 ** -24 * umax
    tau = eps * umax
    band = np.abs(np.abs(pk) - tau) <= 1e-5 * tau + 64 * 2.0 ** -24 * umax
    band[: 1 << (2 * om.coarsest_level(p))] = False
    assert np.array_equal(gmask[~band], mask[~band])


@pytest.mark.parametrize("p,J", [(2, 4), (2, 7), (3, 6)])
def test_inverse_fp64_bitexact(M, p, J):
    N = 1 << J
    pk = om.forward(_field(N, 1), J, p)
    g = M.grid_desc(J, p, 0.0)
    out = torch.empty((N, N), dtype=torch.float64, device=DEV)
    M.mra_transform(g, M.MRA_FP64, M.MRA_INVERSE, _t(pk), out)
    assert np.array_equal(out.cpu().numpy(), om.inverse(pk, J, p))


def _active_inputs(u, J, p, eps):
    pk = om.forward(u, J, p)
    mask, ip, fi = om.threshold(pk, u, eps, J, p)
    return mask, ip, fi


@pytest.mark.parametrize("p,J,eps", [(2, 5, 1e-3), (2, 8, 1e-4), (3, 7, 1e-3), (2, 6, 0.0), (2, 9, 1e-4),
                                     (3, 9, 1e-3), (2, 10, 1e-3), (3, 8, 0.0), (2, 11, 1e-3), (3, 11, 1e-3),
                                     (3, 11, 1e-2), (2, 10, 0.0), (3, 11, 3e-4)])
@pytest.mark.parametrize("prec", [0, 1])
def test_prolong(M, p, J, eps, prec):
    """Pi at every node against the oracle: FP64 bit-exact, FP32 within 2e-6
    of the scale.  J = 11 takes the largest grid, where the coarse levels'
    pair offsets vary from tile to tile; (2, 10, 0) and (3, 11, 3e-4) have
    more than half of the nodes active, where tiles whose every node is active
    skip the level sweep (all of them at eps = 0, some at 3e-4)."""
    N = 1 << J
    u = _field(N, 4)
    mask, ip, fi = _active_inputs(u, J, p, eps)
    vals = W.random_field(N, 17).ravel()[fi]
    g = M.grid_desc(J, p, eps)
    dt = M.bulk_dtype(prec)
    out = torch.empty((N, N), dtype=dt, device=DEV)
    M.mra_transform(g, prec, M.MRA_PROLONG, _t(vals), out, _t(mask, torch.uint8), None,
                    _t(fi, torch.int32), _t(np.array([fi.size]), torch.int64))
    got = out.cpu().numpy().astype(np.float64)
    if prec == M.MRA_FP64:
        assert np.array_equal(got, om.prolong(vals, fi, J, p))
    else:
        ref = om.prolong(vals.astype(np.float32).astype(np.float64), fi, J, p)
        assert np.abs(got - ref).max() <= 2e-6 * np.abs(ref).max()


def _gpu_rhs(M, g, fl, prec, mask, fi, omega, v=None):
    n = fi.size
    out = torch.empty(n, dtype=torch.float64, device=DEV)
    M.collocation_rhs(g, fl, prec, _t(mask, torch.uint8), _t(fi, torch.int32),
                      _t(np.array([n]), torch.int64), _t(omega), None if v is None else _t(v), out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("p,J,eps", [(2, 5, 1e-3), (2, 7, 1e-4), (3, 6, 1e-3), (3, 7, 0.0), (2, 4, 0.0),
                                     (2, 8, 1e-4)])
@pytest.mark.parametrize("smag", [2, 0])
def test_rhs_and_jvp_fp64(M, p, J, eps, smag):
    N = 1 << J
    h = 2 * math.pi / N
    u = _field(N, 5, noise=1e-2)
    mask, ip, fi = _active_inputs(u, J, p, eps)
    omega = u.ravel()[fi]
    nu0 = 1e-3
    fl = oo.Flow(nu0=nu0, cs=0.17, mu=0.05, smag_mode=smag)
    g = M.grid_desc(J, p, eps)
    gf = M.flow_desc(nu0, 0.17, 0.0, 0.05, smag)
    wt = om.prolong(omega, fi, J, p)
    base = oo.base_fields(wt, h, p, fl)
    F = oo.rhs(wt, h, p, fl, base).ravel()[fi]
    got = _gpu_rhs(M, g, gf, M.MRA_FP64, mask, fi, omega)
    sc = max(np.abs(F).max(), np.abs(oo.advection(base["u"], base["v"], wt, h, p)).max())
    assert np.abs(got - F).max() <= 1e-10 * sc
    v = W.random_field(N, 23, smooth=1).ravel()[fi]
    Jv = oo.jvp(om.prolong(v, fi, J, p), base, h, p, fl).ravel()[fi]
    gotv = _gpu_rhs(M, g, gf, M.MRA_FP64, mask, fi, omega, v)
    assert np.abs(gotv - Jv).max() <= 1e-10 * np.abs(Jv).max()


@pytest.mark.parametrize("p,J,eps", [(2, 7, 1e-4), (3, 6, 1e-3)])
def test_rhs_and_jvp_fp32(M, p, J, eps):
    N = 1 << J
    h = 2 * math.pi / N
    u = _field(N, 6, noise=1e-2)
    mask, ip, fi = _active_inputs(u, J, p, eps)
    omega = u.ravel()[fi].astype(np.float32).astype(np.float64)
    fl = oo.Flow(nu0=1e-3, cs=0.17)
    g = M.grid_desc(J, p, eps)
    gf = M.flow_desc(1e-3, 0.17)
    wt = om.prolong(omega, fi, J, p)
    base = oo.base_fields(wt, h, p, fl)
    F = oo.rhs(wt, h, p, fl, base).ravel()[fi]
    adv = oo.advection(base["u"], base["v"], wt, h, p).ravel()[fi]
    dif = oo.diffusion(base["nu"], wt, h, p).ravel()[fi]
    sc = max(np.abs(F).max(), np.abs(adv).max(), np.abs(dif).max())
    got = _gpu_rhs(M, g, gf, M.MRA_MIXED, mask, fi, omega)
    assert np.abs(got - F).max() <= 2e-5 * sc
    v = W.random_field(N, 29, smooth=1).ravel()[fi].astype(np.float32).astype(np.float64)
    vt = om.prolong(v, fi, J, p)
    Jv = oo.jvp(vt, base, h, p, fl).ravel()[fi]
    gotv = _gpu_rhs(M, g, gf, M.MRA_MIXED, mask, fi, omega, v)
    # the same scale rule as for F: the largest of the product and its
    # advective and diffusive parts (they cancel in J v as in F)
    uv, vv = oo.velocities(oo.poisson(vt, h, p), h, p)
    adv_v = -(oo.d1(uv * wt + base["u"] * vt, 1, h, p) + oo.d1(vv * wt + base["v"] * vt, 0, h, p))
    scv = max(np.abs(Jv).max(), np.abs(adv_v.ravel()[fi]).max(),
              np.abs(oo.diffusion(base["nu"], vt, h, p).ravel()[fi]).max())
    errF, errJ = np.abs(got - F).max() / sc, np.abs(gotv - Jv).max() / scv
    print(f"FP32 J={J} p={p}: F err {errF:.2e}, J v err {errJ:.2e} (of the scale; bar 2e-5)")
    assert errJ <= 2e-5


def _solve_pair(M, pb, prec, m=None, dt=None):
    g = M.grid_desc(pb.J, pb.p, pb.eps)
    f = M.flow_desc(pb.nu0, pb.cs)
    w0 = W.initial_field(pb)
    return M.Solve(g, f, prec, m or pb.m, dt or pb.dt, _t(w0)), w0


def _oracle_run(pb, w0, nsteps, m=None, dt=None):
    g = ok.Grid(J=pb.J, p=pb.p, eps=pb.eps)
    fl = oo.Flow(nu0=pb.nu0, cs=pb.cs)
    st = ok.init_state(w0, g)
    for _ in range(nsteps):
        st = ok.step(st, g, fl, m or pb.m, dt or pb.dt)
    return st, g


def test_solve_init_matches_oracle(M):
    pb = W.plain_pair()
    s, w0 = _solve_pair(M, pb, M.MRA_FP64)
    om_, mask, ip, fi = s.active_set()
    st, g = _oracle_run(pb, w0, 0)
    assert np.array_equal(mask.cpu().numpy(), st.mask)
    assert np.array_equal(fi.cpu().numpy(), st.index_fine)
    assert np.array_equal(om_.cpu().numpy(), st.omega_M)


@pytest.mark.parametrize("nsteps", [1, 4])
def test_step_fp64_matches_oracle(M, nsteps):
    pb = W.plain_pair()
    s, w0 = _solve_pair(M, pb, M.MRA_FP64)
    s.step(nsteps)
    dense, diag = s.read()
    st, g = _oracle_run(pb, w0, nsteps)
    ref = om.prolong(st.omega_M, st.index_fine, pb.J, pb.p)
    got = dense.cpu().numpy()
    _, mask, _, fi = s.active_set()
    assert np.array_equal(mask.cpu().numpy(), st.mask)
    assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)
    d = ok.diagnostics(ref, g)
    assert abs(diag["energy"] - d["energy"]) <= 1e-10 * d["energy"]
    assert abs(diag["enstrophy"] - d["enstrophy"]) <= 1e-10 * d["enstrophy"]
    assert abs(diag["t"] - nsteps * pb.dt) < 1e-12
    assert int(diag["n_active"]) == st.omega_M.size


def test_step_fp64_fine_levels_matches_oracle(M):
    # J = 8: the prolongation runs its fused fine-level kernel
    pb = W.fujiwhara_pair(1003, J=8)
    s, w0 = _solve_pair(M, pb, M.MRA_FP64, m=12)
    s.step(2)
    dense, diag = s.read()
    st, g = _oracle_run(pb, w0, 2, m=12)
    ref = om.prolong(st.omega_M, st.index_fine, pb.J, pb.p)
    _, mask, _, _ = s.active_set()
    assert np.array_equal(mask.cpu().numpy(), st.mask)
    assert np.linalg.norm(dense.cpu().numpy() - ref) <= 1e-10 * np.linalg.norm(ref)


def test_step_mixed_error_reported(M):
    pb = W.plain_pair()
    s, w0 = _solve_pair(M, pb, M.MRA_MIXED)
    s.step(3)
    dense, diag = s.read()
    st, g = _oracle_run(pb, w0, 3)
    ref = om.prolong(st.omega_M, st.index_fine, pb.J, pb.p)
    rel = np.linalg.norm(dense.cpu().numpy() - ref) / np.linalg.norm(ref)
    d = ok.diagnostics(ref, g)
    print(f"mixed vs oracle after 3 steps: rel L2 {rel:.3e}, dE/E {abs(diag['energy'] - d['energy']) / d['energy']:.3e}")
    assert rel <= 1e-5


def test_batch_equals_alone(M):
    pbs = [W.plain_pair(), W.fujiwhara_pair(1001, J=6), W.fujiwhara_pair(1000, J=7), W.plain_pair(J=5)]
    alone = []
    for pb in pbs:
        s, _ = _solve_pair(M, pb, M.MRA_MIXED, m=10)
        s.step(2)
        alone.append(s.read()[0].cpu().numpy())
        s.close()
    solves = [_solve_pair(M, pb, M.MRA_MIXED, m=10)[0] for pb in pbs]
    M.solve_batch(solves, [2] * len(solves))
    for s, a in zip(solves, alone):
        assert np.array_equal(s.read()[0].cpu().numpy(), a)


def test_stream_batch_equals_alone(M):
    """17 equal-configuration solves advanced together on a stream (captured
    step graphs); solve 0 stops a step early, so the batch changes
    composition.  Every solve is bit-identical to the same solve stepped alone
    with krylov_step on the same stream."""
    pbs = [W.fujiwhara_pair(2000 + i, J=6) for i in range(17)]
    steps = [2] + [3] * 16
    st = torch.cuda.Stream(device=DEV)

    def make(pb):
        with torch.cuda.stream(st):
            w0 = _t(W.initial_field(pb))
            return M.Solve(M.grid_desc(pb.J, pb.p, pb.eps), M.flow_desc(pb.nu0, pb.cs), M.MRA_MIXED, 12, pb.dt,
                           w0, stream=st)

    alone = []
    for pb, k in zip(pbs, steps):
        s = make(pb)
        s.step(k, stream=st)
        alone.append(s.read(stream=st)[0].cpu().numpy())
        s.close()
    solves = [make(pb) for pb in pbs]
    M.solve_batch(solves, steps, stream=st)
    for s, a in zip(solves, alone):
        assert np.array_equal(s.read(stream=st)[0].cpu().numpy(), a)
    for s in solves:
        s.close()


def test_uneven_stream_batch_equals_alone(M):
    """Solves of three grid sizes, two precisions and a passive scalar advanced
    by one solve_batch call on a stream: each step of the whole batch is one
    captured graph whose branches are the configuration groups (the scalar's
    branch after its partner's).  Uneven step counts change the composition
    mid-call.  Every solve is bit-identical to the same solve stepped alone."""
    pbs = [W.fujiwhara_pair(3000, J=5), W.fujiwhara_pair(3001, J=6), W.fujiwhara_pair(3002, J=7),
           W.fujiwhara_pair(3003, J=6)]
    precs = [M.MRA_MIXED, M.MRA_MIXED, M.MRA_FP64, M.MRA_MIXED]
    steps = [3, 2, 3, 3]
    st = torch.cuda.Stream(device=DEV)

    def make(pb, prec):
        with torch.cuda.stream(st):
            return M.Solve(M.grid_desc(pb.J, pb.p, pb.eps), M.flow_desc(pb.nu0, pb.cs), prec, 8, pb.dt,
                           _t(W.initial_field(pb)), stream=st)

    def scalar(partner, pb):
        with torch.cuda.stream(st):
            return M.ScalarSolve(partner, M.grid_desc(pb.J, pb.p, 1e-3), 8, pb.dt,
                                 _t(W.vapor_field(pb.N, 4.0)), eddy=True, stream=st)

    alone = []
    for pb, prec, k in zip(pbs, precs, steps):
        s = make(pb, prec)
        sc = scalar(s, pb) if pb is pbs[3] else None
        for _ in range(k):
            s.step(1, stream=st)
            if sc is not None:
                sc.step(1, stream=st)
        alone.append(s.read(stream=st)[0].cpu().numpy())
        if sc is not None:
            alone.append(sc.read(stream=st)[0].cpu().numpy())
            sc.close()
        s.close()
    solves = [make(pb, prec) for pb, prec in zip(pbs, precs)]
    sc = scalar(solves[3], pbs[3])
    handles = solves + [sc]
    M.solve_batch(handles, steps + [steps[3]], stream=st)
    got = [h.read(stream=st)[0].cpu().numpy() for h in solves] + [sc.read(stream=st)[0].cpu().numpy()]
    for i, (g_, a) in enumerate(zip(got, alone)):
        assert np.array_equal(g_, a), f"solve {i} differs"
    sc.close()
    for s in solves:
        s.close()

"""GPU parity at the lengths and shapes of the benchmark configurations,
against the FP64 oracle on the same seeded inputs.

* The plain configuration (two Gaussians, r0 = 0.3, centres (pi -/+ 0.6, pi),
  64^2, 4-point DD, eps 1e-3, Re 5000, Cs 0.17, m = 20, dt = 0.01) over its
  full 100 steps in FP64: the active set bit-exact at every 10th step; the
  vorticity, energy and enstrophy within 1e-10 at the end.
* The three-vortex Re = 37440 configuration's shape (6-point DD, eps 1e-4,
  m = 30, dt = 0.002, white noise of amplitude 1e-3, every node active at
  first) on 512^2 over two steps and on 1024^2 over one, in FP64 (bit-exact
  masks, 1e-10), and in mixed precision (1e-5, mask flips counted).
"""
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


def _solve(M, pb, prec):
    w0 = W.initial_field(pb)
    s = M.Solve(M.grid_desc(pb.J, pb.p, pb.eps), M.flow_desc(pb.nu0, pb.cs), prec, pb.m, pb.dt,
                torch.from_numpy(w0).to(DEV))
    return s, w0


def _compare(M, s, st, g):
    """(rel L2 of the vorticity, dE/E, dZ/Z, mask flips, GPU status) of a
    solve against an oracle state."""
    dense, diag = s.read()
    ref = om.prolong(st.omega_M, st.index_fine, g.J, g.p)
    got = dense.cpu().numpy()
    d = ok.diagnostics(ref, g)
    _, mask, _, _ = s.active_set()
    return (float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
            abs(diag["energy"] - d["energy"]) / d["energy"],
            abs(diag["enstrophy"] - d["enstrophy"]) / d["enstrophy"],
            int((mask.cpu().numpy() != st.mask).sum()), int(diag["status"]), diag)


def test_plain_pair_full_length_fp64(M):
    pb = W.plain_pair()
    assert (pb.J, pb.steps, pb.m, pb.dt, pb.eps) == (6, 100, 20, 0.01, 1e-3)
    s, w0 = _solve(M, pb, M.MRA_FP64)
    g = ok.Grid(J=pb.J, p=pb.p, eps=pb.eps)
    fl = oo.Flow(nu0=pb.nu0, cs=pb.cs)
    st = ok.init_state(w0, g)
    for k in range(10, pb.steps + 1, 10):
        s.step(10)
        for _ in range(10):
            st = ok.step(st, g, fl, pb.m, pb.dt)
        _, mask, _, fi = s.active_set()
        assert np.array_equal(mask.cpu().numpy(), st.mask), f"active set differs after {k} steps"
        assert np.array_equal(fi.cpu().numpy(), st.index_fine), f"index list differs after {k} steps"
    rel, dE, dZ, flips, status, diag = _compare(M, s, st, g)
    print(f"plain pair 64^2 FP64, {pb.steps} steps: rel L2 {rel:.2e}, dE/E {dE:.2e}, dZ/Z {dZ:.2e}, "
          f"N_a {st.omega_M.size}")
    assert status == 0 and flips == 0
    assert abs(diag["t"] - pb.steps * pb.dt) < 1e-10
    assert rel <= 1e-10 and dE <= 1e-10 and dZ <= 1e-10
    s.close()


@pytest.fixture(scope="module")
def three512():
    """The three-vortex configuration's shape at 512^2: the oracle's two steps."""
    pb = dataclasses.replace(W.three_vortex(), J=9)
    w0 = W.initial_field(pb)
    g = ok.Grid(J=pb.J, p=pb.p, eps=pb.eps)
    fl = oo.Flow(nu0=pb.nu0, cs=pb.cs)
    states = [ok.init_state(w0, g)]
    for _ in range(2):
        states.append(ok.step(states[-1], g, fl, pb.m, pb.dt))
    return pb, g, states


def test_three_vortex_shape_512_fp64(M, three512):
    pb, g, states = three512
    assert (pb.p, pb.m, pb.dt, pb.eps, pb.noise_amp) == (3, 30, 0.002, 1e-4, 1e-3)
    s, _ = _solve(M, pb, M.MRA_FP64)
    _, mask, _, _ = s.active_set()
    assert np.array_equal(mask.cpu().numpy(), states[0].mask)
    for k in (1, 2):
        s.step(1)
        rel, dE, dZ, flips, status, _ = _compare(M, s, states[k], g)
        print(f"three vortices 512^2 FP64, step {k}: rel L2 {rel:.2e}, dE/E {dE:.2e}, dZ/Z {dZ:.2e}, "
              f"N_a {states[k].omega_M.size} ({states[k].omega_M.size / pb.N ** 2:.1%})")
        assert status == 0 and flips == 0
        assert rel <= 1e-10 and dE <= 1e-10 and dZ <= 1e-10
    s.close()


def test_three_vortex_shape_512_mixed(M, three512):
    pb, g, states = three512
    s, _ = _solve(M, pb, M.MRA_MIXED)
    s.step(2)
    rel, dE, dZ, flips, status, _ = _compare(M, s, states[2], g)
    print(f"three vortices 512^2 mixed, 2 steps: rel L2 {rel:.2e}, dE/E {dE:.2e}, dZ/Z {dZ:.2e}, "
          f"mask flips {flips} of {states[2].omega_M.size}")
    assert status == 0
    assert rel <= 1e-5 and dE <= 1e-5 and dZ <= 1e-5
    assert flips <= 1e-3 * states[2].omega_M.size
    s.close()


def test_three_vortex_shape_1024_fp64(M):
    pb = dataclasses.replace(W.three_vortex(), J=10)
    s, w0 = _solve(M, pb, M.MRA_FP64)
    g = ok.Grid(J=pb.J, p=pb.p, eps=pb.eps)
    st = ok.step(ok.init_state(w0, g), g, oo.Flow(nu0=pb.nu0, cs=pb.cs), pb.m, pb.dt)
    s.step(1)
    rel, dE, dZ, flips, status, _ = _compare(M, s, st, g)
    print(f"three vortices 1024^2 FP64, 1 step: rel L2 {rel:.2e}, dE/E {dE:.2e}, N_a {st.omega_M.size}")
    assert status == 0 and flips == 0
    assert rel <= 1e-10 and dE <= 1e-10 and dZ <= 1e-10
    s.close()

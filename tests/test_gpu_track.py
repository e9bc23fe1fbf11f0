"""GPU vortex-centre tracking (Section 3.2) against the oracle's rule on the
same field: one update from offset guesses, and a tracked 128^2 Fujiwhara run
(every step) against the oracle update applied to the GPU's field."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import track as otr
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
    w0 = torch.from_numpy(W.initial_field(pb)).to(DEV)
    return M.Solve(M.grid_desc(pb.J, pb.p, pb.eps), M.flow_desc(pb.nu0, pb.cs), prec, pb.m, pb.dt, w0)


def test_track_matches_oracle_rule(M):
    pb = W.fujiwhara_pair(1000, J=7)
    s = _solve(M, pb, M.MRA_FP64)
    dense, _ = s.read()
    guess = [(v.cx + 0.07, v.cy - 0.05) for v in pb.vortices]
    got = s.track(guess)
    ref = otr.update_centres(dense.cpu().numpy(), guess)
    assert np.allclose(got, ref, rtol=0, atol=1e-12)
    s.close()


def test_tracked_run_matches_oracle_rule(M):
    pb = W.fujiwhara_pair(1001, J=7)
    s = _solve(M, pb, M.MRA_MIXED)
    cg = [(v.cx, v.cy) for v in pb.vortices]
    co = list(cg)
    b0 = otr.separation(*cg)
    for _ in range(20):
        s.step(1)
        dense, _ = s.read()
        co = otr.update_centres(dense.cpu().numpy(), cg)
        cg = s.track(cg)
        assert np.allclose(cg, co, rtol=0, atol=1e-12)
    b = otr.separation(*cg)
    print(f"tracked 20 steps: b/b0 = {b / b0:.6f}, t* = {20 * pb.dt / otr.convective_time(b0, 1.0):.4f}")
    assert 0.5 < b / b0 < 1.5
    s.close()
